"""The oracle's pins, checked against plausible mistakes in the oracle itself.

Each case below plants one mistake in a copy of ``oracle/cv_oracle.c`` (a
wrong tie order, a dropped term, a transposed operand, an off-by-one in a
comparison), compiles the copy on the CPU, and runs the pins of
``test_oracle_pins.py`` that should catch it against that copy.  A mutant
that no pin rejects fails the test: a pin set that would let that mistake
through is not a pin.
"""
import os

import pytest

import oracle
import test_oracle_pins as pins

# (name, text in cv_oracle.c, its replacement, the pins that must reject it)
MUTANTS = [
    ("merge takes the right run on equal keys",
     "if (key_less(a[j], a[i])) tmp[k++] = a[j++];", "if (!key_less(a[i], a[j])) tmp[k++] = a[j++];",
     ["test_sort_matches_lexsort_with_ties", "test_sort_brute_force_tiny"]),
    ("sort ignores the time stamp",
     "    return g_ts[i] < g_ts[j];\n}\n\n/* sort a[lo, hi)", "    return 0;\n}\n\n/* sort a[lo, hi)",
     ["test_sort_matches_lexsort_with_ties"]),
    ("sort compares ids as unsigned",
     "if (g_jid[i] != g_jid[j]) return g_jid[i] < g_jid[j];\n    return g_ts[i]",
     "if (g_jid[i] != g_jid[j]) return (uint64_t)g_jid[i] < (uint64_t)g_jid[j];\n    return g_ts[i]",
     ["test_sort_signed_extremes"]),
    ("haversine without cos(phi1)",
     "double a = (sp * sp) + ((cphi1 * cphi2) * (sl * sl));", "double a = (sp * sp) + ((cphi2) * (sl * sl));",
     ["test_one_degree_of_meridian_and_equator", "test_haversine_and_bearing_vs_mpmath"]),
    ("radius in kilometres",
     "static const double EARTH_R_M = 6371008.8;", "static const double EARTH_R_M = 6371.0088;",
     ["test_one_degree_of_meridian_and_equator"]),
    ("bearing with atan2 operands swapped",
     "b = atan2(y, x) * RAD2DEG;", "b = atan2(x, y) * RAD2DEG;",
     ["test_cardinal_bearings"]),
    ("bearing x term with the wrong sign of the correction",
     "double x = sin(dphi) + (((2.0 * sin(phi1)) * cphi2) * (sl * sl));",
     "double x = sin(dphi) - (((2.0 * sin(phi1)) * cphi2) * (sl * sl));",
     ["test_long_steps_vs_mpmath"]),
    ("heading change wrapped into [-180, 180)",
     "else if (d <= -180.0) d += 360.0;", "else if (d < -180.0) d += 360.0;",
     ["test_heading_change_wrap"]),
    ("acceleration over the predecessor's speed reversed",
     "acc = (v - speed_mps[p]) / dts;", "acc = (speed_mps[p] - v) / dts;",
     ["test_dt_speed_accel_on_meridian_walk"]),
    ("no zero-dt flag",
     "unsigned f = (dt_ms == 0) ? F_DT_ZERO : 0u;", "unsigned f = 0u;",
     ["test_flags_heads_duplicates_and_bad_coordinates"]),
    ("journey head ignores the id change",
     "int head = (k == 0) || (jid[k] != jid[k - 1]);", "int head = (k == 0);",
     ["test_flags_heads_duplicates_and_bad_coordinates"]),
    ("summary sums without the half-way correction",
     "        if (y == yr) hi = x;\n", "",
     ["test_fsum_cancellation_and_halfway"]),
    ("negative zero kept in the bounding box",
     "double a = lat[i] + 0.0, o = lon[i] + 0.0;", "double a = lat[i], o = lon[i];",
     ["test_summary_bbox_signed_zero_and_no_finite_points"]),
    ("max derived speed over every point",
     "if ((flags[i] & F_SPEED_OK) && dspeed[i] > maxd) maxd = dspeed[i];", "if (dspeed[i] > maxd) maxd = dspeed[i];",
     ["test_summary_max_derived_speed_only_over_speed_ok"]),
    ("grid key with latitude and longitude transposed",
     "key[i] = (tb * n_lat + (int64_t)fy) * n_lon + (int64_t)fx;",
     "key[i] = (tb * n_lat + (int64_t)fx) * n_lon + (int64_t)fy;",
     ["test_grid_brute_force"]),
    ("time bin by truncating division",
     "    if ((a % b != 0) && ((a < 0) != (b < 0))) q -= 1;\n    return q;\n}\n\nint64_t orc_grid_keys",
     "    return q;\n}\n\nint64_t orc_grid_keys",
     ["test_grid_line_cases"]),
    ("a journey counted once per record",
     "if (c == a || jid[i] != jid[idx[c - 1]]) ++nj;", "++nj;",
     ["test_grid_brute_force", "test_grid_distinct_journeys_with_cell_reentry"]),
    ("late when equal to the newest earlier time",
     "if (have_last && ts[i] < last) {", "if (have_last && ts[i] <= last) {",
     ["test_stream_late_by_hand"]),
    ("a late record moves the journey's last point back to itself",
     "                late[i] = 1;\n                ++n_late;\n",
     "                late[i] = 1;\n                ++n_late;\n                last = ts[i];\n",
     ["test_stream_late_by_hand"]),
    ("history forgotten after a push with only late records",
     "                have_cur = 0;\n                cur_push = push[i];",
     "                if (!have_cur) have_last = 0;\n                have_cur = 0;\n                cur_push = push[i];",
     ["test_stream_late_by_hand"]),
]


def _run_pin(name):
    """Run the named pin (all its parametrisations); True when every case passes."""
    fn = getattr(pins, name)
    marks = getattr(fn, "pytestmark", [])
    params = [m for m in marks if m.name == "parametrize"]
    if not params:
        try:
            fn(oracle)
            return True
        except AssertionError:
            return False
    argnames, values = params[0].args[0], params[0].args[1]
    names = [a.strip() for a in argnames.split(",")]
    for v in values:
        v = v if isinstance(v, tuple) else (v,)
        try:
            fn(oracle, **dict(zip(names, v)))
        except AssertionError:
            return False
    return True


@pytest.mark.parametrize("name,old,new,pin_names", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_pins_reject_mutant(oracle_mod, tmp_path, name, old, new, pin_names):
    src = open(oracle.SRC).read()
    assert src.count(old) == 1, f"mutation site not unique or missing: {old!r}"
    mut = tmp_path / "mutant.c"
    mut.write_text(src.replace(old, new))
    so = oracle.compile_to(str(mut), str(tmp_path / "libmutant.so"))
    saved = oracle._lib
    oracle._lib = oracle.bind(so)
    try:
        caught = [p for p in pin_names if not _run_pin(p)]
    finally:
        oracle._lib = saved
    assert caught, f"no pin rejects the mutant '{name}' (tried {pin_names})"


def test_unmutated_oracle_passes_the_same_pins(oracle_mod):
    for p in sorted({p for m in MUTANTS for p in m[3]}):
        assert _run_pin(p), p
