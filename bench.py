#!/usr/bin/env python
"""Benchmark of the connected-vehicle ETL path on one MI355X.

One step = the whole hot path over one batch resident in HBM: stable sort by
(journey, time) with key-then-payload gather, per-point kinematics, per-journey
summaries and the (time bin x cell) group table.

The default run measures, in one JSON line:
  * the headline: the plain path on the full-day Missouri-shaped synthetic day
    (50 000 journeys, lognormal lengths with median 1 500 points, 5 %
    duplicated and 2 % swapped timestamps, 0.005 deg x 5 min grid), about
    124 M records -- Mrecords/s (median of per-step HIP events), the roofline
    of the dominant kernel (radix scatter pass) measured with HIP events on its
    launch stream, the whole path's algorithmic bytes over the step time, and
    the CPU oracle timed on a bounded sample of the same workload;
  * "batched": 115 county-day shards of capped Zipf sizes (400 M records,
    0.001 deg x 1 min) in one set of launches, against the plain path called
    per shard on the same resident input, with every shard's outputs compared;
  * "serving": a Poisson stream of 200 chunks/s (10 k - 5 M records) served
    with continuous batching and one chunk per push on the identical trace:
    p50 / p95 / p99 chunk latency and Mrecords/s, outputs compared.
--workload c0|c1|c2|c3|c4 runs one of them on its own.
"""
from __future__ import annotations

import argparse
import ctypes
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="all", choices=["all", "c0", "c1", "c2", "c3", "c4"])
    ap.add_argument("--duration", type=float, default=None, help="c3/c4: seconds of arrivals")
    ap.add_argument("--shards", type=int, default=115, help="c2: number of shards")
    ap.add_argument("--total", type=int, default=400_000_000, help="c2: total records")
    ap.add_argument("--n-journeys", type=int, default=None, help="scale the workload down (testing)")
    ap.add_argument("--no-direction", action="store_true", help="c1: skip the direction-lattice measurement")
    ap.add_argument("--separate", action="store_true",
                    help="run the sort and the kinematics as two calls instead of the fused one")
    ap.add_argument("--cpu-sample", type=int, default=40_000_000, help="records in the oracle's timed sample")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-batched", action="store_true", help="default run: skip the batched sub-benchmark")
    ap.add_argument("--no-serving", action="store_true", help="default run: skip the serving sub-benchmark")
    ap.add_argument("--c4-rates", type=lambda x: [float(v) for v in x.split(",")], default=[200.0, 400.0, 600.0, 800.0],
                    help="c4: constant chunk rates of the sustained-rate sweep")
    ap.add_argument("--sweep-duration", type=float, default=6.0, help="c4: seconds per sweep rate")
    ap.add_argument("--push-records", type=int, default=None,
                    help="c3/c4: most records one push batches (default: a quarter of the ring)")
    ap.add_argument("--batched-steps", type=int, default=5, help="default run: timed steps of the batched form")
    ap.add_argument("--batched-only", action="store_true",
                    help="c2: time the batched form only (no per-shard loop or comparison; for profiler runs)")
    ap.add_argument("--out", default=None, help="also write the JSON line to this file")
    ap.add_argument("--sort-shape", type=int, default=None,
                    help="radix tile shape index (default: the tuning cache, else the library default)")
    ap.add_argument("--copy-calibration", type=int, default=None, metavar="MIB",
                    help="only run a plain device copy of MIB MiB five times (the known-size reference "
                         "for the HBM byte counters) and exit")
    return ap.parse_args()


def copy_calibration(mib):
    """A plain device-to-device copy of a known size: read mib MiB, write mib MiB
    per launch.  Profiled with FETCH_SIZE / WRITE_SIZE, it gives the factor
    between those counters and bytes moved."""
    import torch
    n = mib * (1 << 20) // 4
    a = torch.rand(n, device="cuda")
    b = torch.empty_like(a)
    torch.cuda.synchronize()
    for _ in range(5):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_calibration_bytes_per_launch": {"read": n * 4, "write": n * 4}, "launches": 5}))


def make_workload(name, n_journeys):
    from paper_2305_07454_amd import gen
    t = time.time()
    if name == "c0":
        r = gen.make_c0(**({"n_journeys": n_journeys} if n_journeys else {}))
        desc = "plain small: 2000 journeys x U{100..900} points, shuffled, 0.01 deg x 15 min"
    else:
        r = gen.make_c1(**({"n_journeys": n_journeys} if n_journeys else {}))
        desc = ("plain full-day: 50000 journeys, lognormal lengths (median 1500, sigma 1, cap 86400) "
                "at 1 Hz, 5% duplicated / 2% swapped timestamps, per-journey files in random order, "
                "0.005 deg x 5 min")
    log(f"generated {name}: {r.n} records in {time.time() - t:.1f}s")
    return r, gen.GRIDS[name], desc


def host_cpu():
    """CPU model and the cores this process may use (the oracle runs on one)."""
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        usable = len(os.sched_getaffinity(0))
    except AttributeError:
        usable = os.cpu_count()
    return model, usable


def cpu_baseline(r, grid, target):
    """The oracle, untuned, single-threaded, on the first journeys (file order)
    of the same workload until `target` records."""
    import numpy as np
    import oracle
    jid = r.journey_id
    # journeys are contiguous blocks in file order (c1); take whole blocks
    change = np.nonzero(jid[1:] != jid[:-1])[0] + 1
    cut = int(change[np.searchsorted(change, min(target, r.n)) - 1]) if r.n > target and len(change) else r.n
    if cut <= 0:
        cut = min(target, r.n)
    cols = tuple(np.ascontiguousarray(c[:cut]) for c in r.columns())
    oracle.lib()
    t = time.perf_counter()
    oracle.run_plain(cols, grid)
    dt = time.perf_counter() - t
    n_j = int(len(np.unique(cols[0])))
    model, usable = host_cpu()
    return {"value": round(cut / dt / 1e6, 4), "unit": "Mrecords/s", "cores": 1, "kind": "oracle",
            "cpu_model": model, "nproc": usable,
            "sample": f"first {n_j} journeys in file order ({cut} records) of the same workload, "
                      f"whole plain path, {dt:.1f}s, one thread"}


def step_stats(ms):
    """Median / min / max / std of per-step times (ms)."""
    import numpy as np
    a = np.asarray(ms, dtype=np.float64)
    return {"median": round(float(np.median(a)), 4), "min": round(float(a.min()), 4),
            "max": round(float(a.max()), 4), "std": round(float(a.std()), 4), "mean": round(float(a.mean()), 4),
            "steps": int(a.size)}


def timed_steps(fn, steps, stream):
    """Run fn() `steps` times with a HIP event pair around each step on
    `stream`; returns the per-step times in ms."""
    import torch
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(steps + 1)]
    ev[0].record(stream)
    for i in range(steps):
        fn()
        ev[i + 1].record(stream)
    torch.cuda.synchronize()
    return [ev[i].elapsed_time(ev[i + 1]) for i in range(steps)]


def _same(a, b):
    import torch
    return a.shape == b.shape and torch.equal(a.contiguous().view(torch.uint8), b.contiguous().view(torch.uint8))


def bench_batched(args, steps):
    """Batched form (all shards in one set of launches) vs the plain path called
    once per shard, same resident input, same GPU; every shard's outputs of the
    two are compared bit for bit."""
    import numpy as np
    import torch
    from paper_2305_07454_amd import cvetl, gen
    dev = torch.device("cuda:0")
    t = time.time()
    shards = gen.make_c2(n_shards=args.shards, total=args.total)
    sizes = [s.n for s in shards]
    allr = gen.concat(shards)
    del shards
    n = allr.n
    log(f"generated c2: {len(sizes)} shards, {n} records in {time.time() - t:.1f}s")
    grid = gen.GRIDS["c2"]
    rec = cvetl.to_device(allr, dev)
    del allr
    torch.cuda.synchronize()
    log(f"c2 columns resident ({time.time() - t:.1f}s)")
    from paper_2305_07454_amd import tune
    tune.apply(n, workload="c2")
    off_h, off_d = cvetl.shard_offsets(sizes, dev)
    bp, res = cvetl.cv_batch_run(rec, sizes, grid)
    J, G = res[1]["count"], res[2]["count"]
    mj = bp.max_journeys
    log(f"sizing run: {J} journeys, {G} groups ({time.time() - t:.1f}s)")
    del bp
    torch.cuda.empty_cache()
    bp = cvetl.BatchPipeline(n, len(sizes), grid, mj, J, max(4096, int(1.25 * G)), dev, fused=not args.separate)
    for _ in range(args.warmup):
        bp.run(rec, off_d)
    torch.cuda.synchronize()
    assert all(x["status"] == 0 for x in bp.results())
    log(f"warm-up done ({time.time() - t:.1f}s)")
    stream = torch.cuda.current_stream()
    cvetl.cv_timing_reset()
    cvetl.cv_timing_enable(True)
    torch.cuda.synchronize()
    per_step = timed_steps(lambda: bp.run(rec, off_d), steps, stream)
    cvetl.cv_timing_enable(False)
    st = step_stats(per_step)
    ms_batched = st["median"]
    rs_b = bp.results()[0]
    roof_b, pass_ms_b = radix_roofline(cvetl, n, rs_b)
    stages_b = {}
    for fam in ("sort_prep", "gather", "features", "gather_features", "summary", "grid_agg", "grid_tail"):
        ms, c = cvetl.cv_timing_read(fam)
        if c:
            stages_b[fam] = round(ms / steps, 4)
    stages_b["sort_passes"] = round(pass_ms_b / steps, 4)
    log(f"batched: {ms_batched:.2f} ms per step (median of {steps}) ({time.time() - t:.1f}s)")
    out = {
        "workload": f"c2: {len(sizes)} county-day shards, capped Zipf(1.2) sizes {min(sizes)}..{max(sizes)}, "
                    f"time-ordered feed per shard, 0.001 deg x 1 min, batched in one set of launches",
        "records": n, "shards": len(sizes), "journeys": J, "groups": G,
        "value": round(n / (ms_batched / 1e3) / 1e6, 3), "unit": "Mrecords/s",
        "ms_per_step": ms_batched, "step_ms": st,
        "roofline": roof_b,
        "stages_ms_per_step": stages_b,
        "path_roofline": path_roofline(stages_b, n, G, rs_b["key_bits"], rs_b["packed_pass"], ms_batched,
                                       design_bytes=317, digit_bits=int(cvetl.cv_tuning_get("radix_bits")),
                                       interleaved=True, ts_in_key=False, first_bits=first_digit_bits(rs_b)),
        "key_bits": rs_b["key_bits"],
        "first_digit_bits": first_digit_bits(rs_b),
        "packed_from_pass": rs_b["packed_pass"],
    }
    if args.batched_only:
        del bp, rec
        torch.cuda.empty_cache()
        return out
    # plain per-file: one plain pipeline sized for the largest shard, called per shard
    big = max(sizes)
    pp = cvetl.Pipeline(big, grid, max_journeys=max(1024, mj), journey_capacity=max(1, J),
                        group_capacity=max(4096, int(1.25 * G)), device=dev, fused=not args.separate)
    views = [{k: v[int(off_h[i]):int(off_h[i + 1])] for k, v in rec.items()} for i in range(len(sizes))]

    def per_file():
        for v in views:
            if v["journey_id"].numel():
                pp.run(v)

    per_file()
    torch.cuda.synchronize()
    pf_steps = max(1, min(steps, 3))
    pf = step_stats(timed_steps(per_file, pf_steps, stream))
    ms_plain = pf["median"]
    log(f"per-file: {ms_plain:.2f} ms per step ({time.time() - t:.1f}s)")
    # identical outputs, every shard: the per-file path once more, compared after each shard
    jo = bp.journey_offsets.cpu().numpy()
    go = bp.group_offsets.cpu().numpy()
    checked = 0
    for i, v in enumerate(views):
        m = int(v["journey_id"].numel())
        if not m:
            continue
        pp.run(v)
        rr = pp.results()
        a, b = int(off_h[i]), int(off_h[i + 1])
        ok = _same(bp.perm[a:b], pp.perm[:m])
        ok = ok and all(_same(bp.sorted[k][a:b], pp.sorted[k][:m]) for k in bp.sorted)
        ok = ok and all(_same(bp.feat[k][a:b], pp.feat[k][:m]) for k in bp.feat)
        ok = ok and int(jo[i + 1] - jo[i]) == rr[1]["count"] and int(go[i + 1] - go[i]) == rr[2]["count"]
        ok = ok and all(_same(bp.journeys[k][int(jo[i]):int(jo[i + 1])], pp.journeys[k][:rr[1]["count"]])
                        for k in bp.journeys)
        ok = ok and all(_same(bp.groups[k][int(go[i]):int(go[i + 1])], pp.groups[k][:rr[2]["count"]])
                        for k in bp.groups)
        assert ok, f"batched and per-file outputs differ on shard {i}"
        checked += 1
    log(f"batched == per-file on all {checked} shards ({time.time() - t:.1f}s)")
    out["plain_per_file"] = {"value": round(n / (ms_plain / 1e3) / 1e6, 3), "ms_per_step": ms_plain, "step_ms": pf,
                             "unit": "Mrecords/s"}
    out["batched_speedup"] = round(ms_plain / ms_batched, 3)
    out["identical_outputs_shards_checked"] = checked
    del bp, pp, rec, views
    torch.cuda.empty_cache()
    return out


def bench_serving(args, workload):
    """Serving at a fixed Poisson arrival rate: continuous batching vs one chunk
    per push on the identical trace; p50/p99 chunk latency and Mrecords/s."""
    import numpy as np
    import torch
    from paper_2305_07454_amd import gen, serve
    skew = workload == "c4"
    t = time.time()
    pool = gen.make_stream(n_journeys=50_000, heavy_frac=0.01 if skew else 0.0, heavy_share=0.3,
                           heavy_cap=500_000, config_index=4 if skew else 3)
    log(f"generated stream pool: {pool.n} records in {time.time() - t:.1f}s")
    grid = gen.GRIDS[workload]
    if skew:
        dur = args.duration or 30.0
        third = dur / 3.0
        rate = lambda tt: 1000.0 if third <= tt < 2 * third else 200.0  # noqa: E731
        desc = (f"serving under skew: 1% of journeys (20 Hz, up to 500k points) hold ~30% of records; "
                f"0.001 deg x 1 min; 200 chunks/s with a 5x burst in the middle third of {dur:.0f}s")
    else:
        dur = args.duration or 10.0
        rate = lambda tt: 200.0  # noqa: E731
        desc = f"serving: Poisson 200 chunks/s for {dur:.0f}s, chunks 10k-5M records (log-uniform); 0.005 deg x 5 min"
    trace = serve.poisson_trace(np.random.default_rng(2024), rate, dur, 10_000, 5_000_000)
    log(f"trace: {len(trace)} chunks, {sum(s for _, s in trace) / 1e6:.0f} M records")
    out = {}
    flushed = {}
    keep = 40
    max_groups = (1 << 26) if skew else (1 << 22)
    arena = None
    for name, batching in (("batched", True), ("per_chunk", False)):
        srv = serve.Server(pool, grid, batching=batching, arena_records=arena, max_journeys=1 << 22,
                           max_groups=max_groups, max_push_records=args.push_records)
        arena = srv.A  # both servers get the arena the first carved from free HBM
        chunks = srv.run(trace, keep_first=keep, log=lambda m: log(f"{name}: {m}"))
        out[name] = serve.latency_stats(chunks, warmup_s=min(2.0, dur / 5))
        log(f"{name}: {out[name]}")
        flushed[name] = (srv.flush(1 << 23, max_groups), srv.keep)
        del srv
        torch.cuda.empty_cache()
    (ja, ga, ra, rga), ka = flushed["batched"]
    (jb, gb, rb, rgb), kb = flushed["per_chunk"]
    same = all(_same(ja[k], jb[k]) for k in ja) and all(_same(ga[k], gb[k]) for k in ga) and \
        all(_same(ka[c][k], kb[c][k]) for c in ka for k in ka[c])
    flags_clear = ra["flags"] == 0 and rb["flags"] == 0
    for nm, rj, rg in (("batched", ra, rga), ("per_chunk", rb, rgb)):
        log(f"{nm}: journeys {rj['count']} status {rj['status']} cell-overflow flag {rj['flags']}; "
            f"groups {rg['count']} status {rg['status']}")
    assert same, "batched and per-chunk serving differ"
    assert flags_clear, "a distinct-journey cell set overflowed: counts may be high"
    offered = sum(s for _, s in trace) / dur / 1e6
    sweep = serving_rate_sweep(pool, grid, arena, max_groups, args.c4_rates, args.sweep_duration,
                               args.push_records) if skew else None
    return {
        "workload": f"{workload}: {desc}", "pool_records": pool.n, "chunks": len(trace),
        "offered_mrec_per_s": round(offered, 1), "arena_records": int(arena),
        "admission": "FIFO into a ring of record slots carved from free HBM at start-up; "
                     f"a push batches at most {args.push_records or 'a quarter of the ring'} records",
        "value": out["batched"]["mrec_per_s"], "unit": "Mrecords/s",
        "latency_batched": out["batched"], "latency_per_chunk": out["per_chunk"],
        "identical_outputs": bool(same and flags_clear), "journeys": int(ra["count"]), "groups": int(rga["count"]),
        "rate_sweep": sweep,
    }


def serving_rate_sweep(pool, grid, arena, max_groups, rates, dur, push_records=None):
    """The batched server at constant Poisson rates (same chunk sizes as the
    burst trace), a fresh server per rate.  A rate is sustained when the
    latency does not grow over the run: the p90 of the last third of the
    chunks stays within twice the p90 of the first third plus 20 ms, and the
    p99 stays below 100 ms."""
    import numpy as np
    import torch
    from paper_2305_07454_amd import serve
    rows = []
    for rate in rates:
        # seeded by the rate itself, so a rate replays the same trace in any list
        trace = serve.poisson_trace(np.random.default_rng(7000 + int(round(rate))), lambda tt, r=rate: r, dur,
                                    10_000, 5_000_000)
        srv = serve.Server(pool, grid, batching=True, arena_records=arena, max_journeys=1 << 22,
                           max_groups=max_groups, max_push_records=push_records)
        chunks = srv.run(trace)
        st = serve.latency_stats(chunks, warmup_s=min(1.0, dur / 5))
        lat = [c.t_done - c.arrival for c in chunks if c.arrival >= min(1.0, dur / 5)]
        k = max(1, len(lat) // 3)
        p90a, p90b = float(np.percentile(lat[:k], 90)), float(np.percentile(lat[-k:], 90))
        ok = p90b <= 2.0 * p90a + 0.02 and st["p99_ms"] < 100.0
        offered = sum(s for _, s in trace) / dur / 1e6
        rows.append({"chunks_per_s": rate, "offered_mrec_per_s": round(offered, 1), "p50_ms": st["p50_ms"],
                     "p99_ms": st["p99_ms"], "mrec_per_s": st["mrec_per_s"], "sustained": bool(ok)})
        log(f"sweep {rate}/s: {rows[-1]}")
        del srv
        torch.cuda.empty_cache()
    best = max((r["chunks_per_s"] for r in rows if r["sustained"]), default=None)
    return {"duration_s": dur, "rates": rows, "highest_sustained_chunks_per_s": best}


def bench_plain(args, workload):
    """The plain path on one resident batch (C1 by default)."""
    import torch
    from paper_2305_07454_amd import cvetl
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    r, grid, desc = make_workload(workload, args.n_journeys)
    n = r.n
    if args.sort_shape is not None:
        cvetl.cv_tuning_set("sort_shape", args.sort_shape)
    else:
        from paper_2305_07454_amd import tune
        tune.apply(n, workload=workload)
    log(f"sort shape {cvetl.cv_tuning_get('sort_shape')} (tile {cvetl.cv_tuning_get('sort_tile')} keys)")
    rec = cvetl.to_device(r, dev)
    torch.cuda.synchronize()

    # size the outputs once (untimed) from a run of the self-sizing calls
    out = cvetl.run_plain(rec, grid)
    J = int(out["summary_result"]["count"])
    G = int(out["grid_result"]["count"])
    del out
    torch.cuda.empty_cache()
    pipe = cvetl.Pipeline(n, grid, max_journeys=max(1024, 2 * J), journey_capacity=J,
                          group_capacity=max(4096, int(1.25 * G)), device=dev, fused=not args.separate)
    log(f"n={n} J={J} G={G} workspace={pipe.workspace_bytes() / 2**30:.2f} GiB"
        f" ({'separate' if args.separate else 'fused'} gather and kinematics)")

    for _ in range(args.warmup):
        pipe.run(rec)
    torch.cuda.synchronize()
    for res in pipe.results():
        assert res["status"] == 0, res

    cvetl.cv_timing_reset()
    cvetl.cv_timing_enable(True)
    stream = torch.cuda.current_stream()
    torch.cuda.synchronize()
    wall = time.perf_counter()
    per_step = timed_steps(lambda: pipe.run(rec), args.steps, stream)
    wall = time.perf_counter() - wall
    cvetl.cv_timing_enable(False)
    st = step_stats(per_step)
    ms_step = st["median"]
    rs, rj, rg = pipe.results()
    assert rs["status"] == 0 and rj["status"] == 0 and rg["status"] == 0

    # invariants on the benchmarked outputs
    npts = pipe.journeys["n_points"][:J].to(torch.int64).sum().item()
    cnt = pipe.groups["count"][:G].to(torch.int64).sum().item()
    assert npts == n, (npts, n)
    assert cnt + rg["n_out_of_grid"] == n, (cnt, rg["n_out_of_grid"], n)

    # dominant kernel: the radix scatter passes that run (digit below the key width)
    key_bits = rs["key_bits"]
    p0 = rs["packed_pass"]
    roof, pass_ms = radix_roofline(cvetl, n, rs)
    stages = {}
    for fam in ("sort_prep", "gather", "features", "gather_features", "summary", "grid_agg", "grid_tail"):
        ms, c = cvetl.cv_timing_read(fam)
        if c:
            stages[fam] = round(ms / args.steps, 4)
    stages["sort_passes"] = round(pass_ms / args.steps, 4)

    direction, lattice = None, None
    if not args.no_direction and workload == "c1":
        direction, gdir = bench_direction(args, r, grid, pipe, rec, G, dev)
        lattice = bench_lattice(args, grid, {k: v[:G] for k, v in pipe.groups.items()}, gdir, dev)
        lattice["hygiene"] = bench_hygiene(pipe, n, dev)
        lattice["csv_extract"] = bench_csv(r, dev)

    traffic = None
    tfile = os.path.join(ROOT, "profiles", "radix_pass_c1_traffic.md")
    if workload == "c1" and args.n_journeys is None and os.path.exists(tfile):
        t = read_traffic(tfile)
        if t.get("kernel_source_sha") == _kernel_sha() and t.get("sort_shape") == str(cvetl.cv_tuning_get("sort_shape")):
            traffic = float(t["traffic_bytes_per_launch"])

    del pipe, rec
    torch.cuda.empty_cache()
    cpu = None
    if not args.no_cpu_baseline:
        log("timing the oracle on a bounded sample")
        cpu = cpu_baseline(r, grid, args.cpu_sample)

    value = n / (ms_step / 1e3) / 1e6
    return {
        "metric": METRIC,
        "value": round(value, 3),
        "unit": "Mrecords/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"{workload}: {desc}", "records": n, "journeys": J, "groups": G,
                   "path": "plain", "parallelism": "single GPU"},
        "step_ms": st,
        "roofline": dict(roof, traffic=traffic),
        "cpu_baseline": cpu,
        "stages_ms_per_step": stages,
        "path_roofline": path_roofline(stages, n, G, key_bits, p0, ms_step,
                                       design_bytes=282 if workload == "c1" else None,
                                       digit_bits=int(cvetl.cv_tuning_get("radix_bits")),
                                       first_bits=first_digit_bits(rs)),
        "direction_lattice": direction,
        "dense_lattice": lattice,
        "key_bits": key_bits,
        "first_digit_bits": first_digit_bits(rs),
        "packed_from_pass": p0,
        "wall_s_timed_region": round(wall, 3),
    }


METRIC = "ETL Mrecords/s & % HBM peak (plain vs batched); serving p50/p99 latency"


def _line(args, sub, workload):
    """A whole JSON line for a sub-benchmark run on its own."""
    path = "batched" if workload == "c2" else "served, continuous batching"
    return {"metric": METRIC, "value": sub["value"], "unit": "Mrecords/s", "n_gpus": 1,
            "steps": sub.get("step_ms", {}).get("steps", sub.get("chunks")), "warmup": args.warmup,
            "ms_per_step": sub.get("ms_per_step", sub.get("latency_batched", {}).get("p50_ms")),
            "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
            "config": {"workload": sub["workload"], "path": path, "parallelism": "single GPU"},
            "roofline": sub.get("roofline"), "cpu_baseline": None, workload: sub}


def main():
    args = parse()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}, WORLD_SIZE={world}): the ETL path "
              "is built and measured on a single MI355X; see the sharding design notes", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2305_07454_amd import cvetl  # noqa: F401  (fails loudly without the HIP library)

    assert torch.cuda.is_available(), "bench needs a GPU"
    if args.copy_calibration:
        return copy_calibration(args.copy_calibration)
    w = args.workload
    if w == "c2":
        line = _line(args, bench_batched(args, args.steps), "c2")
    elif w in ("c3", "c4"):
        line = _line(args, bench_serving(args, w), w)
    else:
        line = bench_plain(args, "c1" if w == "all" else w)
        if w == "all":
            if not args.no_batched:
                line["batched"] = bench_batched(args, args.batched_steps)
            if not args.no_serving:
                line["serving"] = bench_serving(args, "c3")
    s = json.dumps(line)
    print(s, flush=True)
    if args.out:
        with open(args.out, "w") as f:
            f.write(s + "\n")


def bench_direction(args, r, grid, pipe, rec, G, dev):
    """The lattice with four direction sectors of a sensor heading column on
    the same sorted records: the heading gathered into sorted order, then the
    aggregate.  Timed with HIP events around each call, after the main run."""
    import numpy as np
    import torch
    from paper_2305_07454_amd import cvetl, gen
    n = r.n
    hd = torch.from_numpy(gen.headings(np.random.default_rng(77), r.journey_id)).to(dev)
    hs = torch.empty_like(hd)
    cap = max(4096, int(2.5 * G))
    out = {k: torch.empty(cap, dtype=dt, device=dev) for k, dt in cvetl.GROUP_FIELDS}
    need = cvetl._size(cvetl.lib().cv_grid_workspace_size, n, ctypes.byref(cvetl._spec_struct(grid)), cap)
    ws = cvetl.workspace(need, dev)
    pipe.run(rec)  # the sorted records and perm of this input
    srt = pipe.sorted
    stream = torch.cuda.current_stream()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
    gms, gth = 0.0, 0.0
    steps = max(3, args.steps // 2)
    for i in range(steps + 1):
        ev[0].record(stream)
        cvetl.cv_gather_column(hd, pipe.perm[:n], out=hs)
        ev[1].record(stream)
        _, res = cvetl.cv_grid_aggregate_dir(srt, grid, 4, 0.0, heading=hs, capacity=cap, sync=False, ws=ws,
                                             out=out)
        ev[2].record(stream)
        torch.cuda.synchronize()
        if i > 0:  # the first round warms up
            gth += ev[0].elapsed_time(ev[1])
            gms += ev[1].elapsed_time(ev[2])
    rd = cvetl.read_result(res)
    assert rd["status"] == 0, rd
    cnt = out["count"][:rd["count"]].to(torch.int64).sum().item()
    assert cnt + rd["n_out_of_grid"] == n, (cnt, rd["n_out_of_grid"], n)
    log(f"direction lattice: {rd['count']} groups, gather {gth / steps:.3f} ms, aggregate {gms / steps:.3f} ms")
    info = {"n_dir": 4, "offset_deg": 0.0, "heading": "sensor column (synthetic whole degrees), gathered",
            "groups": rd["count"], "gather_ms": round(gth / steps, 4), "aggregate_ms": round(gms / steps, 4),
            "steps": steps}
    return info, {k: v[:rd["count"]] for k, v in out.items()}


def bench_lattice(args, grid, groups, gdir, dev):
    """Dense lattice of every time bin (mean speed and volume channels per
    sector), its per-channel normalisation, and the group filter, on the full-day
    workload's group tables without and with four sectors.  HIP events around each call."""
    import torch
    from paper_2305_07454_amd import cvetl
    stream = torch.cuda.current_stream()
    n_t = int(grid.n_t)
    res = {}
    for name, g, nd in (("plain", groups, 0), ("four_sectors", gdir, 4)):
        C = cvetl.lattice_channels(nd)
        lat = torch.empty((n_t, C, int(grid.n_lat), int(grid.n_lon)), dtype=torch.float32, device=dev)
        mm = torch.empty(2 * C, dtype=torch.float32, device=dev)
        nws = cvetl.workspace(cvetl._size(cvetl.lib().cv_lattice_normalize_workspace_size, n_t,
                                          ctypes.byref(cvetl._spec_struct(grid)), nd), dev)
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
        dms, nms = 0.0, 0.0
        steps = 3
        for i in range(steps + 1):
            ev[0].record(stream)
            cvetl.cv_lattice_dense(g, grid, nd, 0, n_t, out=lat)
            ev[1].record(stream)
            cvetl.cv_lattice_normalize(lat, grid, nd, minmax=mm, ws=nws)
            ev[2].record(stream)
            torch.cuda.synchronize()
            if i > 0:
                dms += ev[0].elapsed_time(ev[1])
                nms += ev[1].elapsed_time(ev[2])
        nbytes = lat.numel() * 4
        dms, nms = dms / steps, nms / steps
        res[name] = {"shape": list(lat.shape), "tensor_gb": round(nbytes / 1e9, 3), "groups": int(g["key"].numel()),
                     "dense_ms": round(dms, 4), "dense_gbs": round(nbytes / dms / 1e6, 1),
                     "normalize_ms": round(nms, 4)}
        log(f"lattice {name}: {res[name]}")
        del lat
        torch.cuda.empty_cache()
    # filter: groups with >= 2 vehicles and mean speed below 10 m/s
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    cvetl.cv_groups_filter(groups, 2, 0.0, 10.0)
    e0.record(stream)
    idx, r = cvetl.cv_groups_filter(groups, 2, 0.0, 10.0)
    e1.record(stream)
    torch.cuda.synchronize()
    res["filter"] = {"predicate": "n_journeys >= 2 and 0 <= mean speed <= 10 m/s", "groups": int(groups["key"].numel()),
                     "kept": r["count"], "ms_incl_result_read": round(e0.elapsed_time(e1), 4)}
    log(f"filter: {res['filter']}")
    return res


def bench_hygiene(pipe, n, dev):
    """Dropping exact duplicate rows and splitting trips at 60 s gaps, on the
    sorted records of the main run (HIP events around each call)."""
    import torch
    from paper_2305_07454_amd import cvetl
    srt = {k: v[:n] for k, v in pipe.sorted.items()}
    stream = torch.cuda.current_stream()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
    cvetl.cv_drop_duplicates(srt, pipe.perm[:n])
    cvetl.cv_split_trips(srt, 60_000)
    ev[0].record(stream)
    _, _, rd = cvetl.cv_drop_duplicates(srt, pipe.perm[:n])
    ev[1].record(stream)
    _, _, rt = cvetl.cv_split_trips(srt, 60_000)
    ev[2].record(stream)
    torch.cuda.synchronize()
    out = {"kept_records": rd["count"], "drop_duplicates_ms_incl_alloc": round(ev[0].elapsed_time(ev[1]), 4),
           "trips_60s": rt["count"], "split_trips_ms_incl_alloc": round(ev[1].elapsed_time(ev[2]), 4)}
    log(f"hygiene: {out}")
    return out


def bench_csv(r, dev, rows=4_000_000):
    """Extraction of Table-1-shaped text (fixed-width rows of the first
    `rows` records of the full-day workload, written by gen.to_csv) into record
    columns."""
    import numpy as np
    import torch
    from paper_2305_07454_amd import cvetl, gen
    m = min(rows, r.n)
    cols = tuple(c[:m] for c in r.columns())
    t0 = time.time()
    text = gen.to_csv(cols, gen.headings(np.random.default_rng(5), cols[0]))
    dt = torch.from_numpy(np.frombuffer(text, dtype=np.uint8).copy()).to(dev)
    log(f"csv sample: {m} rows, {len(text) / 1e6:.1f} MB generated in {time.time() - t0:.1f}s")
    out, hd, ok, res = cvetl.cv_csv_extract(dt, capacity=m)
    ws = cvetl.workspace(cvetl._size(cvetl.lib().cv_csv_workspace_size, len(text), m), dev)
    stream = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    steps = 5
    e0.record(stream)
    for _ in range(steps):
        cvetl.cv_csv_extract(dt, capacity=m, out=out, heading=hd, row_ok=ok, ws=ws, sync=False)
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / steps
    r2 = cvetl.cv_csv_extract(dt, capacity=m, out=out, heading=hd, row_ok=ok, ws=ws)[3]
    assert r2["count"] == m and r2["n_bad"] == 0, r2
    info = {"rows": m, "text_mb": round(len(text) / 1e6, 1), "ms": round(ms, 4),
            "text_gbs": round(len(text) / ms / 1e6, 1), "mrows_per_s": round(m / ms / 1e3, 1)}
    log(f"csv: {info}")
    return info


def radix_roofline(cvetl, n, rs, traffic=None):
    """Roofline of the record sort's radix scatter passes from the per-pass
    HIP-event timing families (working passes only: digits below the key
    width)."""
    key_bits = rs["key_bits"]
    db = int(cvetl.cv_tuning_get("radix_bits"))
    w0 = first_digit_bits(rs)
    passes = sort_pass_count(key_bits, w0, db)
    p0 = rs["packed_pass"]
    pass_ms, launches, alg = 0.0, 0, 0.0
    per_pass = []
    for p in range(passes):
        ms, c = cvetl.cv_timing_read(f"sort_pass{p}")
        pass_ms += ms
        launches += c
        alg += n * pass_bytes(p, p0) * c
        per_pass.append(round(ms / max(c, 1), 4))
    avg_ms = pass_ms / max(launches, 1)
    per_launch = alg / max(launches, 1)
    achieved = per_launch / (avg_ms / 1e3) / 1e9 if avg_ms > 0 else 0.0
    kind = f"stable {db}-bit LSD scatter pass" if w0 == db else f"stable LSD scatter pass: a {w0}-bit first digit, then {db}-bit digits"
    return {"bound": "hbm", "kernel": f"k_radix_pass ({kind})",
            "tile_keys": cvetl.cv_tuning_get("sort_tile"),
            "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
            "avg_launch_ms": round(avg_ms, 5), "launches": launches,
            "alg_bytes_per_launch": int(per_launch), "per_pass_ms": per_pass}, pass_ms


def first_digit_bits(rs):
    """Bits of the record sort's first radix digit (the sort result's flags
    word: 9 where a key of 8k + 1 bits saves a pass, else 8)."""
    return int(rs.get("flags") or 8)


def sort_pass_count(key_bits, first_bits=8, digit_bits=8):
    """Working radix passes of a key: the first digit first_bits wide, the
    others digit_bits."""
    if key_bits <= 0:
        return 0
    if key_bits <= first_bits:
        return 1
    return 1 + (key_bits - first_bits + digit_bits - 1) // digit_bits


def path_roofline(stages, n, G, key_bits, p0, ms_step, design_bytes=None, digit_bits=8, interleaved=False,
                  ts_in_key=True, first_bits=8):
    """Algorithmic bytes of the whole path per step (the per-record figures of
    each stage's kernels, plus the group tail) over the measured step time.
    design_bytes: the fixed per-record byte budget of the path's design (the
    same for any implementation of it), reported beside as a second fraction.
    interleaved: input with short runs of equal ids, for which the key packing
    also writes a 32-byte payload per record that the fused gather reads
    instead of the columns.  ts_in_key: the sort key holds the time offset."""
    passes = sort_pass_count(key_bits, first_bits, digit_bits)
    # the time offset survives in the final word only when nothing was dropped
    ts_read = 0 if (p0 == 0 and ts_in_key) else 8
    per = {"sort_prep": 16 + 24 + ((20 + 32) if interleaved and "gather_features" in stages else 0),
           "sort_passes": sum(pass_bytes(p, p0) for p in range(passes))}
    if "gather_features" in stages:
        per["gather_features"] = 8 + (32 if interleaved else ts_read + 20) + 4 + 36 + 49
    else:
        per["gather"] = 8 + ts_read + 20 + 4 + 36
        per["features"] = 32 + 49
    per["summary"] = 1 + 17 + 21  # flags for the counts; box pass lat, lon, flags; sums' pass step, speeds, flags
    per["grid_agg"] = 36
    total = n * sum(per.values()) + 64 * G
    gbs = total / (ms_step / 1e3) / 1e9
    out = {"bound": "hbm", "alg_bytes_per_record": per, "group_tail_bytes_per_group": 64,
           "alg_bytes_per_step": int(total), "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
           "frac": round(gbs / HBM_PEAK_GBS, 4)}
    if design_bytes:
        dg = design_bytes * n / (ms_step / 1e3) / 1e9
        out["design_bytes_per_record"] = design_bytes
        out["design_frac"] = round(dg / HBM_PEAK_GBS, 4)
    return out


def pass_bytes(p, p0):
    """Algorithmic bytes per record of radix pass p when passes p0.. move packed
    (key | index) words: read and write 8-byte words, plus 4-byte index values
    before packing (pass 0 generates its indices instead of reading them)."""
    if p >= p0:
        return 16
    rd = 8 + (0 if p == 0 else 4)
    wr = 8 + (0 if p + 1 >= p0 else 4)
    return rd + wr


def read_traffic(path):
    """`key: value` lines of a traffic summary (HBM bytes per radix pass launch
    from the FETCH_SIZE / WRITE_SIZE counters, scaled by a copy of known size)."""
    out = {}
    for line in open(path):
        if ":" in line and not line.startswith(("#", "|", " ", "`")):
            k, v = line.split(":", 1)
            out[k.strip()] = v.strip()
    return out


def _kernel_sha():
    import hashlib
    h = hashlib.sha256()
    for f in ("cv_radix.h", "cv_radix.hip", "cv_device.h"):
        with open(os.path.join(ROOT, "paper_2305_07454_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


if __name__ == "__main__":
    main()
