"""Comparators between the HIP path and the oracle (test helper, not a test).

Bars: orders, keys, counts, flags, integer and exact-summed fields bit-exact;
haversine-derived doubles within 1e-12 relative (glibc and the GPU's libm may
differ by an ulp in sin/asin/atan2); acceleration relative to its operands'
scale; angles on the circle within 1e-12 * 360 degrees.
"""
import numpy as np

REL = 1e-12
ANG = 1e-12 * 360.0


def host(t):
    return t.detach().cpu().numpy()


def u32(a):
    return np.asarray(a).view(np.uint32) if np.asarray(a).dtype == np.int32 else np.asarray(a)


def assert_exact(name, got, exp):
    got = np.asarray(got)
    exp = np.asarray(exp)
    assert got.shape == exp.shape, f"{name}: shape {got.shape} vs {exp.shape}"
    if got.dtype.kind == "f":
        ok = (got.view(np.uint64 if got.itemsize == 8 else np.uint32) ==
              exp.astype(got.dtype).view(np.uint64 if got.itemsize == 8 else np.uint32))
    else:
        ok = got == exp
    if not np.all(ok):
        i = int(np.argmin(ok))
        raise AssertionError(f"{name}: {int((~ok).sum())} mismatches, first at {i}: {got[i]!r} vs {exp[i]!r}")


def assert_rel(name, got, exp, rel=REL):
    got = np.asarray(got, dtype=np.float64)
    exp = np.asarray(exp, dtype=np.float64)
    assert got.shape == exp.shape, name
    err = np.abs(got - exp)
    ok = err <= rel * np.abs(exp)
    if not np.all(ok):
        i = int(np.argmin(ok))
        raise AssertionError(f"{name}: {int((~ok).sum())} beyond {rel} rel, first at {i}: {got[i]!r} vs {exp[i]!r}")


def assert_angle(name, got, exp, tol=ANG):
    d = np.abs(np.asarray(got) - np.asarray(exp))
    d = np.minimum(d, 360.0 - d)
    if not np.all(d <= tol):
        i = int(np.argmax(d))
        raise AssertionError(f"{name}: max circular error {d[i]!r} at {i}")


def check_sort(perm, srt, exp_perm, exp_sorted):
    assert_exact("perm", u32(host(perm)), exp_perm)
    for (k, _), e in zip((("journey_id", 0), ("ts_ms", 0), ("lat_deg", 0), ("lon_deg", 0), ("speed_mps", 0)),
                         exp_sorted):
        assert_exact(f"sorted.{k}", host(srt[k]), e)


def check_features(feat, exp):
    g = {k: host(v) for k, v in feat.items()}
    assert_exact("flags", g["flags"], exp["flags"])
    assert_exact("dt_s", g["dt_s"], exp["dt_s"])
    assert_rel("step_m", g["step_m"], exp["step_m"])
    assert_rel("speed_mps", g["speed_mps"], exp["speed_mps"])
    # acceleration: a difference of two speeds turns one-ulp noise in each into
    # an error relative to the operands, not to the (possibly tiny) difference
    prev = np.concatenate([[0.0], exp["speed_mps"][:-1]])
    dt = np.where(exp["dt_s"] > 0, exp["dt_s"], 1.0)
    scale = (np.abs(exp["speed_mps"]) + np.abs(prev)) / dt
    err = np.abs(g["accel_mps2"] - exp["accel_mps2"])
    assert np.all(err <= REL * scale + 0.0), f"accel: max err {err.max()!r}"
    assert_angle("bearing_deg", g["bearing_deg"], exp["bearing_deg"])
    assert_angle("dheading_deg", g["dheading_deg"], exp["dheading_deg"])


def check_summary(summ, exp):
    g = {k: host(v) for k, v in summ.items()}
    for k in ("journey_id", "t_start_ms", "t_end_ms", "lat_min", "lat_max", "lon_min", "lon_max",
              "max_speed", "sum_speed"):
        assert_exact(f"journeys.{k}", g[k], exp[k])
    for k in ("first", "n_points", "n_dt_zero"):
        assert_exact(f"journeys.{k}", u32(g[k]), exp[k])
    assert_rel("journeys.distance_m", g["distance_m"], exp["distance_m"])
    assert_rel("journeys.max_derived_speed", g["max_derived_speed"], exp["max_derived_speed"])


def check_groups(groups, n_out, exp, exp_out):
    g = {k: host(v) for k, v in groups.items()}
    assert n_out == exp_out, f"n_out_of_grid {n_out} vs {exp_out}"
    assert_exact("groups.key", g["key"], exp["key"])
    for k in ("count", "n_journeys"):
        assert_exact(f"groups.{k}", u32(g[k]), exp[k])
    for k in ("sum_speed", "min_speed", "max_speed"):
        assert_exact(f"groups.{k}", g[k], exp[k])
