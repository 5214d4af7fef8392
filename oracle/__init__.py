"""CPU oracle for the connected-vehicle ETL hot path -- TEST INFRASTRUCTURE.

Only the test suite, ``__graft_entry__.smoke()`` and the benchmark's
``cpu_baseline`` leg may import this package.  The product path (the HIP
library and its binding) never imports it.

The arithmetic lives in ``cv_oracle.c`` (plain single-threaded C, built with
``-ffp-contract=off``); this module marshals numpy arrays and applies the
per-journey gathers.  ``build()`` compiles the C file in place.

Parity status of each function (what pins it is in ``tests/test_oracle_pins.py``):

* ``sort``      -- pinned (numpy.lexsort, brute force over permutations, and a
  mutation check: the merge is the only place ties are ordered)
* ``stream_late`` -- pinned (hand-worked pushes, invariants: one push or
  per-journey non-decreasing times give no late record)
* ``features``  -- pinned (closed forms, mpmath 50-digit references, identities)
* ``summary``   -- pinned (math.fsum, numpy reductions, invariants)
* ``grid``      -- pinned (brute-force Python dict, explicit grid-line cases)
* ``fsum``      -- pinned (math.fsum)
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "cv_oracle.c")
LIB = os.path.join(HERE, "libcvoracle.so")

FLAG_FIRST, FLAG_DT_ZERO, FLAG_SPEED_OK, FLAG_ACCEL_OK = 0x01, 0x02, 0x04, 0x08
FLAG_BEARING_OK, FLAG_DHEAD_OK, FLAG_BAD_COORD = 0x10, 0x20, 0x40

_lib = None


CFLAGS = ["-O2", "-std=c11", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared"]


def compile_to(src: str, out: str, extra=()) -> str:
    """gcc the oracle source `src` into the shared library `out`."""
    tmp = out + ".tmp"
    subprocess.check_call(["gcc", *CFLAGS, *extra, "-o", tmp, src, "-lm"])
    os.replace(tmp, out)
    return out


def build(force: bool = True) -> str:
    """Compile the oracle (gcc, -O2, no FMA contraction, no fast-math)."""
    if force or not os.path.exists(LIB):
        compile_to(SRC, LIB)
    return LIB


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
            build()
        _lib = bind(LIB)
    return _lib


def bind(path):
    """Load a compiled oracle library and declare its C signatures."""
    L = ctypes.CDLL(path)
    P = ctypes.c_void_p
    I = ctypes.c_int64
    D = ctypes.c_double
    L.orc_fsum.argtypes = [I, P]
    L.orc_fsum.restype = D
    L.orc_sort.argtypes = [I, P, P, P]
    L.orc_sort.restype = None
    L.orc_stream_late.argtypes = [I, P, P, I, P, P]
    L.orc_stream_late.restype = I
    L.orc_features.argtypes = [I] + [P] * 11
    L.orc_features.restype = None
    L.orc_summary.argtypes = [I] + [P] * 8 + [I] + [P] * 14
    L.orc_summary.restype = I
    L.orc_grid_keys.argtypes = [I, P, P, P, D, D, D, D, I, I, I, I, I, P]
    L.orc_grid_keys.restype = I
    L.orc_grid.argtypes = [I, P, P, P, P, P, D, D, D, D, I, I, I, I, I, I] + [P] * 7
    L.orc_grid.restype = I
    L.orc_dir_sector.argtypes = [D, ctypes.c_int32, I, D]
    L.orc_dir_sector.restype = I
    L.orc_grid_dir.argtypes = [I] + [P] * 8 + [I, D, D, D, D, D, I, I, I, I, I, I] + [P] * 7
    L.orc_grid_dir.restype = I
    return L


def _p(a):
    return a.ctypes.data_as(ctypes.c_void_p)


def _c(a, dt):
    return np.ascontiguousarray(a, dtype=dt)


def fsum(x) -> float:
    x = _c(x, np.float64)
    return float(lib().orc_fsum(x.shape[0], _p(x)))


def sort(jid, ts):
    """Stable order of record indices by (journey id, timestamp)."""
    jid = _c(jid, np.int64)
    ts = _c(ts, np.int64)
    n = jid.shape[0]
    perm = np.empty(n, dtype=np.uint32)
    lib().orc_sort(n, _p(jid), _p(ts), _p(perm))
    return perm


def stream_late(jid, ts, push_sizes):
    """Late records of a stream pushed in consecutive pieces of `push_sizes`
    records (arrival order): a record is late when its time stamp is below the
    largest time stamp of its journey's non-late records in earlier pushes.
    Returns a bool array over the records in arrival order."""
    jid = _c(jid, np.int64)
    ts = _c(ts, np.int64)
    n = jid.shape[0]
    ends = np.cumsum(np.asarray(push_sizes, dtype=np.int64)).astype(np.int64)
    assert ends.size == 0 or ends[-1] == n, "push sizes must cover the records"
    late = np.zeros(n, dtype=np.uint8)
    lib().orc_stream_late(n, _p(jid), _p(ts), ends.shape[0], _p(ends), _p(late))
    return late.astype(bool)


def sorted_records(cols, perm):
    """Apply the permutation to the five record columns."""
    return tuple(np.ascontiguousarray(c[perm]) for c in cols)


def features(jid, ts, lat, lon):
    jid, ts = _c(jid, np.int64), _c(ts, np.int64)
    lat, lon = _c(lat, np.float64), _c(lon, np.float64)
    n = jid.shape[0]
    out = {k: np.empty(n, dtype=np.float64) for k in
           ("step_m", "dt_s", "speed_mps", "accel_mps2", "bearing_deg", "dheading_deg")}
    out["flags"] = np.empty(n, dtype=np.uint8)
    lib().orc_features(n, _p(jid), _p(ts), _p(lat), _p(lon), _p(out["step_m"]), _p(out["dt_s"]),
                       _p(out["speed_mps"]), _p(out["accel_mps2"]), _p(out["bearing_deg"]),
                       _p(out["dheading_deg"]), _p(out["flags"]))
    return out


SUMMARY_FIELDS = (("journey_id", np.int64), ("first", np.uint32), ("n_points", np.uint32),
                  ("t_start_ms", np.int64), ("t_end_ms", np.int64), ("distance_m", np.float64),
                  ("sum_speed", np.float64), ("max_speed", np.float32),
                  ("max_derived_speed", np.float64), ("n_dt_zero", np.uint32),
                  ("lat_min", np.float64), ("lat_max", np.float64), ("lon_min", np.float64),
                  ("lon_max", np.float64))


def summary(jid, ts, lat, lon, speed, feat):
    jid, ts = _c(jid, np.int64), _c(ts, np.int64)
    lat, lon, speed = _c(lat, np.float64), _c(lon, np.float64), _c(speed, np.float32)
    step = _c(feat["step_m"], np.float64)
    dsp = _c(feat["speed_mps"], np.float64)
    fl = _c(feat["flags"], np.uint8)
    n = jid.shape[0]
    cap = max(1, n)
    out = {k: np.empty(cap, dtype=t) for k, t in SUMMARY_FIELDS}
    J = lib().orc_summary(n, _p(jid), _p(ts), _p(lat), _p(lon), _p(speed), _p(step), _p(dsp), _p(fl),
                          cap, *[_p(out[k]) for k, _ in SUMMARY_FIELDS])
    return {k: v[:J].copy() for k, v in out.items()}


GRID_FIELDS = (("key", np.int64), ("count", np.uint32), ("n_journeys", np.uint32),
               ("sum_speed", np.float64), ("min_speed", np.float32), ("max_speed", np.float32))


def _spec_args(spec):
    return (float(spec.lat0_deg), float(spec.lon0_deg), float(spec.dlat_deg), float(spec.dlon_deg),
            int(spec.n_lat), int(spec.n_lon), int(spec.t0_ms), int(spec.bin_ms), int(spec.n_t))


def grid_keys(ts, lat, lon, spec):
    ts = _c(ts, np.int64)
    lat, lon = _c(lat, np.float64), _c(lon, np.float64)
    n = ts.shape[0]
    key = np.empty(n, dtype=np.int64)
    n_out = lib().orc_grid_keys(n, _p(ts), _p(lat), _p(lon), *_spec_args(spec), _p(key))
    return key, int(n_out)


def grid(jid, ts, lat, lon, speed, spec):
    jid, ts = _c(jid, np.int64), _c(ts, np.int64)
    lat, lon, speed = _c(lat, np.float64), _c(lon, np.float64), _c(speed, np.float32)
    n = jid.shape[0]
    cap = max(1, n)
    out = {k: np.empty(cap, dtype=t) for k, t in GRID_FIELDS}
    n_out = np.zeros(1, dtype=np.int64)
    G = lib().orc_grid(n, _p(jid), _p(ts), _p(lat), _p(lon), _p(speed), *_spec_args(spec), cap,
                       *[_p(out[k]) for k, _ in GRID_FIELDS], _p(n_out))
    res = {k: v[:G].copy() for k, v in out.items()}
    return res, int(n_out[0])


def run_plain(cols, spec):
    """The whole plain path on one batch: order, features, summaries, grid."""
    jid, ts, lat, lon, speed = cols
    perm = sort(jid, ts)
    s = sorted_records(cols, perm)
    feat = features(s[0], s[1], s[2], s[3])
    summ = summary(*s, feat)
    groups, n_out = grid(*s, spec)
    return dict(perm=perm, sorted=s, features=feat, summary=summ, groups=groups, n_out=n_out)


def dir_sector(h, ok, n_dir, offset=0.0):
    """Direction sector of one heading (Algorithm 2's floor division by the
    sector width, read as nd sectors of 360/nd degrees; nd = no direction)."""
    return int(lib().orc_dir_sector(float(h), 1 if ok else 0, int(n_dir), float(offset)))


def grid_dir(jid, ts, lat, lon, speed, spec, n_dir, offset=0.0, heading=None, bearing=None, flags=None):
    """The lattice with a direction dimension: groups keyed by
    ((tbin * (n_dir + 1) + sector) * n_lat + ilat) * n_lon + ilon, the sector
    from `heading` (float32 per record) or else `bearing` with `flags`."""
    jid, ts = _c(jid, np.int64), _c(ts, np.int64)
    lat, lon, speed = _c(lat, np.float64), _c(lon, np.float64), _c(speed, np.float32)
    n = jid.shape[0]
    if heading is not None:
        hd, br, fl = _c(heading, np.float32), None, None
    else:
        hd, br, fl = None, _c(bearing, np.float64), _c(flags, np.uint8)
    cap = max(1, n)
    out = {k: np.empty(cap, dtype=t) for k, t in GRID_FIELDS}
    n_out = np.zeros(1, dtype=np.int64)
    nullp = ctypes.c_void_p(0)
    G = lib().orc_grid_dir(n, _p(jid), _p(ts), _p(lat), _p(lon), _p(speed),
                           _p(hd) if hd is not None else nullp, _p(br) if br is not None else nullp,
                           _p(fl) if fl is not None else nullp, int(n_dir), float(offset), *_spec_args(spec),
                           cap, *[_p(out[k]) for k, _ in GRID_FIELDS], _p(n_out))
    res = {k: v[:G].copy() for k, v in out.items()}
    return res, int(n_out[0])


# ---------------------------------------------------------------------------
# dense lattice, normalisation, filter (plain numpy definitions)
# ---------------------------------------------------------------------------

def lattice_dense(groups, spec, n_dir, t_first, n_t):
    """Methods steps (4)-(5) and the transformed-data output: the group table
    scattered into a dense [n_t][C][n_lat][n_lon] float32 tensor, C = 2 D
    (D = n_dir + 1 sectors, or 1 without directions).  Channel 2 d: mean
    sensor speed of sector d (sum / count in double, rounded to float32);
    channel 2 d + 1: distinct journeys (volume).  Empty cells are 0."""
    D = n_dir + 1 if n_dir else 1
    n_lat, n_lon = int(spec.n_lat), int(spec.n_lon)
    cells = n_lat * n_lon
    out = np.zeros((n_t, 2 * D, n_lat, n_lon), dtype=np.float32)
    key = np.asarray(groups["key"], dtype=np.int64)
    td, cell = key // cells, key % cells
    tb, d = td // D, td % D
    t = tb - t_first
    m = (key >= 0) & (t >= 0) & (t < n_t)
    cnt = np.asarray(groups["count"], dtype=np.float64)[m]
    mean = np.where(cnt > 0, np.asarray(groups["sum_speed"], dtype=np.float64)[m] / np.where(cnt > 0, cnt, 1.0), 0.0)
    iy, ix = cell[m] // n_lon, cell[m] % n_lon
    out[t[m], 2 * d[m], iy, ix] = mean.astype(np.float32)
    out[t[m], 2 * d[m] + 1, iy, ix] = np.asarray(groups["n_journeys"], dtype=np.float64)[m].astype(np.float32)
    return out


def lattice_normalize(lat):
    """Table 2's normalisation rows, read as min-max per channel over all time
    bins: an occupied cell (its sector's volume > 0) becomes
    (x - min) / (max - min) over that channel's occupied cells (double,
    rounded to float32; 0 when max == min); empty cells stay 0.  Returns the
    new tensor and the [C][2] min / max (NaN for a channel with no occupied
    cell)."""
    out = lat.copy()
    C = lat.shape[1]
    mm = np.full((C, 2), np.nan, dtype=np.float32)
    for c0 in range(0, C, 2):
        occ = lat[:, c0 + 1] > 0
        for c in (c0, c0 + 1):
            x = lat[:, c][occ]
            if x.size == 0:
                continue
            mn, mx = x.min(), x.max()
            mm[c] = (mn, mx)
            if mx > mn:
                y = ((x.astype(np.float64) - np.float64(mn)) / (np.float64(mx) - np.float64(mn))).astype(np.float32)
            else:
                y = np.zeros_like(x)
            ch = out[:, c]
            ch[occ] = y
    return out, mm


def groups_filter(groups, min_volume, speed_lo, speed_hi):
    """Table 2's filter row, read as a predicate over groups: ascending indices
    of the groups with distinct journeys >= min_volume and mean speed
    (sum / count) in [speed_lo, speed_hi]."""
    cnt = np.asarray(groups["count"], dtype=np.float64)
    nj = np.asarray(groups["n_journeys"], dtype=np.float64)
    mean = np.asarray(groups["sum_speed"], dtype=np.float64) / np.where(cnt > 0, cnt, 1.0)
    keep = (cnt > 0) & (nj >= min_volume) & (mean >= speed_lo) & (mean <= speed_hi)
    return np.flatnonzero(keep).astype(np.int64)


# ---------------------------------------------------------------------------
# record hygiene (plain Python definitions)
# ---------------------------------------------------------------------------

def drop_duplicates(sorted_cols):
    """Exact duplicate rows (Table 1's first and fourth rows are one): in
    (journey, time)-sorted records, a record is dropped when an earlier record
    of the same (journey id, time stamp) has bit-identical latitude, longitude
    and speed.  Returns the sorted positions of the records kept."""
    jid, ts, lat, lon, spd = sorted_cols
    la = np.ascontiguousarray(lat, dtype=np.float64).view(np.uint64)
    lo = np.ascontiguousarray(lon, dtype=np.float64).view(np.uint64)
    sp = np.ascontiguousarray(spd, dtype=np.float32).view(np.uint32)
    keep = []
    seen = set()
    for k in range(len(jid)):
        if k == 0 or jid[k] != jid[k - 1] or ts[k] != ts[k - 1]:
            seen = set()
        row = (int(la[k]), int(lo[k]), int(sp[k]))
        if row not in seen:
            keep.append(k)
            seen.add(row)
    return np.array(keep, dtype=np.int64)


def split_trips(jid, ts, gap_ms):
    """Trips of (journey, time)-sorted records: a new trip at a journey's first
    record and after a time gap of more than gap_ms.  Returns (trip number of
    every record, journey id of every trip)."""
    n = len(jid)
    start = np.zeros(n, dtype=bool)
    for k in range(n):
        start[k] = k == 0 or jid[k] != jid[k - 1] or int(ts[k]) - int(ts[k - 1]) > gap_ms
    trip = np.cumsum(start) - 1
    return trip.astype(np.int64), np.asarray(jid, dtype=np.int64)[start]


# ---------------------------------------------------------------------------
# text extraction (plain Python definition of the accepted row shape)
# ---------------------------------------------------------------------------

import calendar as _calendar
import datetime as _datetime
import re as _re

_DEC = _re.compile(rb"^[-+]?([0-9]+\.?[0-9]*|\.[0-9]+)$")
_TS = _re.compile(rb"^([0-9]{4})-([0-9]{2})-([0-9]{2}) ([0-9]{2}):([0-9]{2}):([0-9]{2})(\.([0-9]{1,3}))?$")


def _decimal(b):
    """A plain decimal whose significant digits form an integer below 2^53,
    with at most 22 fraction digits: the double nearest to it; else None."""
    if not _DEC.match(b):
        return None
    body = b.lstrip(b"+-")
    ip, _, fp = body.partition(b".")
    if int((ip + fp) or b"0") >= 1 << 53 or len(fp) > 22:
        return None
    return float(b)


def _timestamp(b):
    m = _TS.match(b)
    if not m:
        return None
    y, mo, d, h, mi, se = (int(m.group(i)) for i in range(1, 7))
    try:
        _datetime.datetime(y, mo, d, h, mi, se)
    except ValueError:
        return None
    frac = m.group(8) or b""
    ms = int(frac.ljust(3, b"0")) if frac else 0
    return _calendar.timegm((y, mo, d, h, mi, se, 0, 0, 0)) * 1000 + ms


def csv_extract(text, has_header=True):
    """Table 1's row shape: journey id (1-8 bytes below 0x80, packed
    big-endian into an int64), timestamp (UTC, optional 1-3 fraction digits,
    in ms), latitude and longitude (doubles), postal code (skipped), speed
    (double rounded to float32), heading (empty -> NaN, else float32).  Lines
    end at LF (a trailing CR is dropped); a last line without LF counts.
    Returns the five record columns, heading, and row_ok (1 for a row of
    that shape; 0 with zero / NaN columns otherwise)."""
    lines = text.split(b"\n")
    if text.endswith(b"\n"):
        lines = lines[:-1]
    if not text:
        lines = []
    if has_header and lines:
        lines = lines[1:]
    n = len(lines)
    jid = np.zeros(n, np.int64)
    ts = np.zeros(n, np.int64)
    lat = np.full(n, np.nan)
    lon = np.full(n, np.nan)
    spd = np.full(n, np.nan, np.float32)
    hd = np.full(n, np.nan, np.float32)
    ok = np.zeros(n, np.uint8)
    for r, line in enumerate(lines):
        if line.endswith(b"\r"):
            line = line[:-1]
        f = line.split(b",")
        if len(f) != 7 or b'"' in line:
            continue
        if not (1 <= len(f[0]) <= 8) or any(c >= 0x80 for c in f[0]):
            continue
        t = _timestamp(f[1])
        la, lo, sp = _decimal(f[2]), _decimal(f[3]), _decimal(f[5])
        h = _decimal(f[6]) if f[6] else float("nan")
        if t is None or la is None or lo is None or sp is None or h is None:
            continue
        jid[r] = int.from_bytes(f[0].ljust(8, b"\x00"), "big")
        ts[r], lat[r], lon[r] = t, la, lo
        spd[r], hd[r] = np.float32(sp), np.float32(h)
        ok[r] = 1
    return (jid, ts, lat, lon, spd), hd, ok
