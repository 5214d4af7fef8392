"""Host logic of bench.py: the algorithmic bytes the roofline figures divide
by (no GPU)."""
import os
import sys

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))

import bench  # noqa: E402


def test_pass_bytes_packed_and_unpacked():
    # packed from the first pass: one 8-byte word in and out per pass
    assert [bench.pass_bytes(p, 0) for p in range(4)] == [16, 16, 16, 16]
    # pass 0 reads keys (indices generated), writes packed words when p0 = 1
    assert bench.pass_bytes(0, 1) == 16
    # unpacked passes carry 4-byte indices: read 8 + 4, write 8 + 4
    assert bench.pass_bytes(0, 3) == 8 + 8 + 4
    assert bench.pass_bytes(1, 3) == 12 + 12
    assert bench.pass_bytes(2, 3) == 12 + 8
    assert bench.pass_bytes(3, 3) == 16


def test_path_roofline_full_day_shape():
    # 43-bit key packed from pass 1, fused gather: with 8-bit digits 6 passes
    # (336 bytes per record), with 9-bit digits 5 passes (320)
    st = {"sort_prep": 1.0, "sort_passes": 1.0, "gather_features": 1.0, "summary": 1.0, "grid_agg": 1.0}
    r8 = bench.path_roofline(st, n=1000, G=10, key_bits=43, p0=1, ms_step=1.0, digit_bits=8)
    assert r8["alg_bytes_per_record"]["sort_passes"] == 96 and sum(r8["alg_bytes_per_record"].values()) == 336
    r = bench.path_roofline(st, n=1000, G=10, key_bits=43, p0=1, ms_step=1.0, digit_bits=9)
    per = r["alg_bytes_per_record"]
    assert per["sort_passes"] == 80 and per["gather_features"] == 125
    assert sum(per.values()) == 320
    assert r["alg_bytes_per_step"] == 1000 * 320 + 64 * 10
    assert abs(r["achieved"] - r["alg_bytes_per_step"] / 1e-3 / 1e9) < 0.1
    assert abs(r["frac"] - r["achieved"] / bench.HBM_PEAK_GBS) < 1e-4


def test_path_roofline_separate_calls_and_time_in_key():
    st = {"gather": 1.0, "features": 1.0}
    r = bench.path_roofline(st, n=1, G=0, key_bits=38, p0=0, ms_step=1.0)
    per = r["alg_bytes_per_record"]
    # the time offset survives in the final word when nothing is dropped
    assert per["gather"] == 8 + 20 + 4 + 36 and per["features"] == 32 + 49
    assert "gather_features" not in per


def test_path_roofline_interleaved_batched_shape():
    # time-ordered shards: 26-bit (shard, rank) key packed from pass 0 (4 passes
    # of 8 bits), the payload packed per record by the key packing and read by
    # the gather instead of the columns
    st = {"sort_prep": 1.0, "sort_passes": 1.0, "gather_features": 1.0, "summary": 1.0, "grid_agg": 1.0}
    r = bench.path_roofline(st, n=1, G=0, key_bits=26, p0=0, ms_step=1.0, digit_bits=8, interleaved=True,
                            ts_in_key=False)
    per = r["alg_bytes_per_record"]
    assert per["sort_prep"] == 16 + 24 + 20 + 32
    assert per["sort_passes"] == 4 * 16
    assert per["gather_features"] == 8 + 32 + 4 + 36 + 49


def test_pass_count_with_a_wide_first_digit():
    # a key of 8k + 1 bits with a 9-bit first digit takes k passes
    assert [bench.sort_pass_count(kb, 9) for kb in (9, 17, 25, 33)] == [1, 2, 3, 4]
    assert [bench.sort_pass_count(kb, 8) for kb in (9, 17, 25, 33)] == [2, 3, 4, 5]
    assert bench.sort_pass_count(0, 9) == 0 and bench.sort_pass_count(8, 9) == 1
    # the sort result's flags word carries the width; 0 (older results) reads as 8
    assert bench.first_digit_bits({"flags": 9}) == 9 and bench.first_digit_bits({"flags": 0}) == 8
    # the full-day key: 33 bits packed from pass 0, four passes of 16 bytes
    st = {"sort_prep": 1.0, "sort_passes": 1.0, "gather_features": 1.0, "summary": 1.0, "grid_agg": 1.0}
    r = bench.path_roofline(st, n=1, G=0, key_bits=33, p0=0, ms_step=1.0, first_bits=9)
    assert r["alg_bytes_per_record"]["sort_passes"] == 4 * 16
    assert sum(r["alg_bytes_per_record"].values()) == 296
