#!/usr/bin/env python3
"""Benchmark of exact (d13, d12, d23)-temporal triangle counting on one MI355X.

Workload: the full-size synthetic graph (directed Chung-Lu, n = 2.6M, 36M static pairs, about
61M temporal edges with a heavy multiplicity tail, bursty timestamps over 7.6 years), deltas
(3600, 3600, 3600).  The edge arrays are loaded into HBM before timing (the load itself is not
timed).  One step is the whole per-graph path: core peel, orientation and store re-layout,
static triangle enumeration, count scheduling, then the count and its reduction.  The value is
temporal edges per second of the timed steps.

Prints one JSON line.  Progress goes to stderr.
"""
from __future__ import annotations

import argparse
import json
import os
import statistics
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


# source file of each event-timed kernel (the HBM traffic measured for a kernel is reported only
# while its source is unchanged since the counters were taken)
# the source files each kernel is compiled from (its .hip file and the library headers it includes);
# a counter record holds the sha256 of their concatenation in this order
_HDR = ["internal.h", "count_dev.h"]
KERNEL_SOURCE = {"peel": ["peel.hip", "internal.h"], "peel_adj": ["peel.hip", "internal.h"],
                 "peel_tail": ["peel.hip", "internal.h"], "core": ["core.hip", "internal.h"],
                 "relayout": ["orient.hip", "internal.h"], "tri_count": ["triangles.hip"] + _HDR,
                 "tri_fill": ["triangles.hip"] + _HDR, "light": ["count.hip"] + _HDR,
                 "medium": ["count.hip"] + _HDR, "unit": ["count.hip"] + _HDR,
                 "heavy_prefix": ["count.hip"] + _HDR, "heavy_count": ["count.hip"] + _HDR,
                 "reduce": ["count.hip"] + _HDR}


def source_sha256(kernel):
    """sha256 of the concatenated source files of `kernel` (KERNEL_SOURCE order)."""
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCE[kernel]:
        h.update(open(os.path.join(ROOT, "paper_2106_02762_amd", "csrc", f), "rb").read())
    return h.hexdigest()
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "hbm_traffic_full_graph.md")


def measured_traffic(kernel):
    """HBM bytes per launch of `kernel` from the committed counter summary (FETCH_SIZE plus
    WRITE_SIZE, scaled by the copy-kernel calibration), or None when there is none for this
    kernel or any of its source files has changed since."""
    if not os.path.exists(TRAFFIC_FILE):
        return None
    # records of "- key: `value`" lines, each starting with its "- kernel:" line
    records, fields = {}, None
    for line in open(TRAFFIC_FILE):
        if line.startswith("- ") and ":" in line:
            k, v = line[2:].split(":", 1)
            k, v = k.strip(), v.strip().strip("`")
            if k == "kernel":
                fields = records.setdefault(v, {})
            if fields is not None:
                fields[k] = v
    fields = records.get(kernel, {})
    if not fields or kernel not in KERNEL_SOURCE:
        return None
    if source_sha256(kernel) != fields.get("source_sha256"):
        return None
    try:
        return int(fields["fetch_bytes_per_launch"]) + int(fields["write_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def count_roofline(st, count_ms, kernels_ms):
    """The count's HBM fraction (wall time of dt_count at the headline delta) under two byte counts:
    the library's (16 bytes per unit triangle: its record is all a unit triangle's count reads) and
    the per-triangle formula that charges every triangle 12 + 36 + 8 (s_uv + s_uw) + 8 min(s_vw,
    probe) bytes (72 for a unit triangle); and beside them the HBM bytes the counters measured for
    the count's kernels (per launch, from the committed summary), when recorded for this source."""
    t = count_ms / 1e3
    n_unit = st["n_unit_triangles"]
    survey = st["alg_bytes"] - st["alg_bytes_unit"] + 72 * n_unit
    parts = ("unit", "light", "medium", "heavy_prefix", "heavy_count")
    measured = {k: measured_traffic(k) for k in parts}
    counter = sum(v for v in measured.values() if v is not None) if all(
        measured[k] is not None for k in ("unit", "light", "medium")) else None
    out = {"kernels_ms": kernels_ms, "count_ms": count_ms,
           "alg_bytes": st["alg_bytes"], "frac": round(st["alg_bytes"] / t / (HBM_PEAK_GBS * 1e9), 4),
           "alg_bytes_per_triangle_formula": survey,
           "frac_per_triangle_formula": round(survey / t / (HBM_PEAK_GBS * 1e9), 4),
           "counter_bytes": counter, "counter_bytes_by_kernel": measured,
           "frac_counter": round(counter / t / (HBM_PEAK_GBS * 1e9), 4) if counter else None,
           "achieved_GBs": round(st["alg_bytes"] / t / 1e9, 2)}
    return out


def run_batched(dt, ctx, k, with_cpu):
    """The batched workload: k independent graphs, each with its own deltas, in one call; every
    result is compared with the same query alone, and every 32nd with the oracle."""
    import synth
    t0 = time.time()
    gs = [synth.batch_graph(i) for i in range(k)]
    deltas = [synth.batch_delta(i) for i in range(k)]
    log(f"generated {k} batch graphs ({sum(g.m for g in gs)} edges) in {time.time() - t0:.1f}s")
    hs = []
    for g in gs:
        h = dt.dt_graph_load(ctx, g.n, g.src, g.dst, g.t)
        dt.dt_graph_build(h)
        hs.append((h, g.n, int(g.t.min()), int(g.t.max())))
    handles = [h for h, *_ in hs]
    qs = [dt.make_query(*d) for d in deltas]
    first = dt.dt_count_batch(ctx, handles, qs)   # the first batch autotunes the item size
    reps = 5
    a = time.perf_counter()
    for _ in range(reps):
        out = dt.dt_count_batch(ctx, handles, qs)
    batch_s = (time.perf_counter() - a) / reps
    a = time.perf_counter()
    alone = [dt.dt_count(h, *d) for h, d in zip(handles, deltas)]
    plain_s = time.perf_counter() - a
    ok = bool((out == first).all()) and all((out[i] == alone[i]).all() for i in range(k))
    oracle_ok = None
    if with_cpu:
        import oracle
        oracle_ok = all(bool((out[i] == oracle.count(gs[i].n, gs[i].src, gs[i].dst, gs[i].t, *deltas[i])).all())
                        for i in range(0, k, 32))
    m = sum(g.m for g in gs)
    res = {"workload": f"{k} directed Chung-Lu graphs, n log-uniform [1e3, 2e5], m = 10 n, own deltas",
           "graphs": k, "edges": m, "batch_ms": round(batch_s * 1e3, 3),
           "plain_one_query_per_launch_ms": round(plain_s * 1e3, 3),
           "speedup_vs_plain": round(plain_s / batch_s, 2),
           "graphs_per_s": round(k / batch_s, 1), "edges_per_s": round(m / batch_s, 1),
           "results_match_alone": ok,
           "item_lengths_tuned": dict(zip(("light", "medium"), dt.dt_ctx_batch_tuning(ctx))),
           "oracle_checked": len(range(0, k, 32)) if with_cpu else 0, "results_match_oracle": oracle_ok}
    log("batched", res)
    return res, hs


def run_served(dt, ctx, graphs, seconds, warmup, rate):
    """Open-loop Poisson stream over resident graphs through the serving loop: p50/p99 latency
    (completion - arrival) after the warm-up, then the burst capacity against one query per
    synchronous launch."""
    import queue
    import threading

    import synth
    spans = [(tmin, tmax) for _, _, tmin, tmax in graphs]
    stream = synth.served_stream(spans, duration_s=warmup + seconds, rate=rate)
    srv = dt.dt_server_start(ctx, max_batch=512, max_inflight_queries=1 << 20)
    ids = [dt.dt_server_add_graph(srv, h) for h, *_ in graphs]
    q = queue.Queue()
    lat, res = {}, {}

    def waiter():
        while True:
            item = q.get()
            if item is None:
                return
            i, ticket, t_arr = item
            r = dt.dt_server_wait(srv, ticket)
            lat[i] = time.perf_counter() - t_arr
            res[i] = r

    ws = [threading.Thread(target=waiter) for _ in range(16)]
    for w in ws:
        w.start()
    t0 = time.perf_counter()
    for i, x in enumerate(stream):
        target = t0 + x["arrival"]
        now = time.perf_counter()
        if target > now:
            time.sleep(target - now)
        t_arr = time.perf_counter()
        ticket = dt.dt_server_submit(srv, ids[x["graph"]], x["d13"], x["d12"], x["d23"], x["t_lo"], x["t_hi"])
        q.put((i, ticket, t_arr))
    for _ in ws:
        q.put(None)
    for w in ws:
        w.join()
    elapsed = time.perf_counter() - t0
    keep = [i for i, x in enumerate(stream) if x["arrival"] >= warmup]
    ls = np.array([lat[i] for i in keep]) * 1e3
    # burst capacity: every query of the measured part submitted at once
    burst = [stream[i] for i in keep]
    a = time.perf_counter()
    tickets = [dt.dt_server_submit(srv, ids[x["graph"]], x["d13"], x["d12"], x["d23"], x["t_lo"], x["t_hi"])
               for x in burst]
    outs = [dt.dt_server_wait(srv, t) for t in tickets]
    burst_s = time.perf_counter() - a
    dt.dt_server_stop(srv)
    # plain comparator: the same queries one synchronous launch each (a prefix of them)
    n_plain = min(len(burst), 3000)
    a = time.perf_counter()
    plain = [dt.dt_count(graphs[x["graph"]][0], x["d13"], x["d12"], x["d23"], x["t_lo"], x["t_hi"])
             for x in burst[:n_plain]]
    plain_s = time.perf_counter() - a
    ok = all((outs[j] == plain[j]).all() for j in range(n_plain)) and \
        all((res[keep[j]] == outs[j]).all() for j in range(len(keep)))
    out = {"workload": f"{len(graphs)} resident graphs (the full-size graph and {len(graphs) - 1} "
                       f"batch-style graphs), Poisson arrivals at {rate:g}/s, deltas as in the batch "
                       "workload, windows log-uniform in [1 day, span]",
           "queries": len(keep), "warmup_s": warmup, "offered_per_s": rate,
           "achieved_per_s": round(len(stream) / elapsed, 1),
           "p50_ms": round(float(np.percentile(ls, 50)), 3), "p99_ms": round(float(np.percentile(ls, 99)), 3),
           "burst_capacity_per_s": round(len(burst) / burst_s, 1),
           "plain_one_query_per_launch_per_s": round(n_plain / plain_s, 1),
           "capacity_vs_plain": round((len(burst) / burst_s) / (n_plain / plain_s), 2),
           "results_match_alone": bool(ok)}
    log("served", out)
    return out


def run_medium(dt, ctx, d, with_cpu):
    """The medium workload (n = 10^6, 10^7 temporal edges, Zipf(2) multiplicity on every pair):
    build + count and count alone on the GPU, whole-span parity with the oracle on all host cores,
    and the oracle's time on one thread (the paper's single-thread setting, as context)."""
    import synth
    t0 = time.time()
    g = synth.plain_medium()
    log(f"generated {g.name}: n={g.n} m={g.m} in {time.time() - t0:.1f}s")
    h = dt.dt_graph_load(ctx, g.n, g.src, g.dst, g.t)
    ts = []
    for _ in range(4):
        a = time.perf_counter()
        dt.dt_graph_build(h)
        out = dt.dt_count(h, d, d, d)
        ts.append((time.perf_counter() - a) * 1e3)
    tc = []
    for _ in range(11):
        a = time.perf_counter()
        dt.dt_count(h, d, d, d)
        tc.append((time.perf_counter() - a) * 1e3)
    st = dt.dt_graph_stats(h)
    res = {"workload": g.name, "n": g.n, "m": g.m, "deltas": [d, d, d],
           "build_count_ms": round(statistics.median(ts[1:]), 3),
           "edges_per_s": round(g.m / (statistics.median(ts[1:]) / 1e3), 1),
           "count_ms": round(statistics.median(tc[1:]), 4),
           "static_triangles": st["n_static_triangles"], "degeneracy": st["degeneracy"],
           "unit": st["n_unit_triangles"], "light": st["n_light_triangles"],
           "medium": st["n_medium_triangles"], "heavy": st["n_heavy_triangles"],
           "counts": out.tolist()}
    if with_cpu:
        import oracle
        threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
        par = {}
        for dd in ((d, d, d), (86400, 86400, 86400), (86400, 3600, 43200)):
            want = oracle.count(g.n, g.src, g.dst, g.t, *dd, nthreads=threads)
            par[",".join(map(str, dd))] = bool((dt.dt_count(h, *dd) == want).all())
        a = time.perf_counter()
        want1 = oracle.count(g.n, g.src, g.dst, g.t, d, d, d, nthreads=1)
        s1 = time.perf_counter() - a
        res["gpu_matches_oracle"] = par
        res["oracle_one_thread"] = {"value": round(g.m / s1, 1), "unit": "temporal edges/s", "cores": 1,
                                    "seconds": round(s1, 3), "matches": bool((want1 == out).all())}
    dt.dt_graph_free(h)
    log("medium", res)
    return res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", choices=["full", "medium"], default="full")
    ap.add_argument("--delta", type=int, default=3600)
    ap.add_argument("--cpu-dottt-frac", type=float, default=0.25,
                    help="CPU DOTTT sample (one thread): edges in the first fraction of the span")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--batch-graphs", type=int, default=512,
                    help="graphs of the batched workload (0 skips the batched and served parts)")
    ap.add_argument("--serve-seconds", type=float, default=60.0)
    ap.add_argument("--no-medium", dest="medium", action="store_false",
                    help="skip the medium workload (10M edges: build + count, oracle parity and timing)")
    ap.add_argument("--serve-warmup", type=float, default=5.0)
    ap.add_argument("--serve-rate", type=float, default=2000.0)
    ap.add_argument("--calib-copy-mib", type=int, default=0,
                    help="first copy this many MiB device to device (calibrates HBM counters)")
    ap.add_argument("--quick", action="store_true",
                    help="only the step and the count at the headline delta (for profiled runs)")
    ap.add_argument("--maps-at-exit", action="store_true",
                    help="write /proc/self/maps to stderr when the interpreter exits (to attribute a "
                         "fault in exit-time teardown to a library)")
    args = ap.parse_args()
    if args.maps_at_exit:
        import atexit

        def _maps():
            sys.stderr.write(open("/proc/self/maps").read())
            sys.stderr.flush()
        atexit.register(_maps)
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU only: the count of one graph runs on a single MI355X "
              "(sharding the triangles over several GPUs is not built); run with --gpus 1",
              file=sys.stderr)
        sys.exit(2)

    import torch

    import paper_2106_02762_amd as dt
    import synth

    t0 = time.time()
    g = synth.plain_full() if args.workload == "full" else synth.plain_medium()
    log(f"generated {g.name}: n={g.n} m={g.m} in {time.time() - t0:.1f}s")
    d = args.delta

    ctx = dt.dt_ctx_create(0)
    dev = torch.device("cuda:0")
    src = torch.from_numpy(g.src.view(np.int32)).to(dev)
    dst = torch.from_numpy(g.dst.view(np.int32)).to(dev)
    tt = torch.from_numpy(g.t).to(dev)
    torch.cuda.synchronize()
    h = dt.dt_graph_load_device(ctx, g.n, src, dst, tt)
    del src, dst, tt
    torch.cuda.synchronize()
    # the timed builds use the default split and kernel geometry: the autotuner's choice among
    # candidates within a few percent of each other varies from run to run (and under a profiler),
    # so the counter records would not match the timed schedule; it is run and reported on its own
    dt.dt_graph_set_tuning(h, autotune=1)
    log("loaded")
    if args.calib_copy_mib > 0:
        a_ = torch.empty(args.calib_copy_mib << 20, dtype=torch.uint8, device=dev)
        b_ = torch.empty_like(a_)
        b_.copy_(a_)
        torch.cuda.synchronize()
        log(f"calibration copy of {args.calib_copy_mib} MiB done")
        del a_, b_
    dt.dt_ctx_set_profiling(ctx, True)

    def step():
        dt.dt_graph_build(h)
        return dt.dt_count(h, d, d, d)

    for _ in range(args.warmup):
        ref = step()
    log("warmup done", ref.tolist())
    prof = []
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    for _ in range(args.steps):
        out = step()
        prof.append(dt.dt_ctx_last_profile(ctx))
    torch.cuda.synchronize()
    t_end = time.perf_counter()
    assert (out == ref).all()
    ms_step = (t_end - t_start) * 1e3 / args.steps
    st = dt.dt_graph_stats(h)
    value = g.m / (ms_step / 1e3)
    log(f"step {ms_step:.2f} ms -> {value:.3e} edges/s")

    if args.quick:
        st = dt.dt_graph_stats(h)
        ts = []
        for _ in range(11):
            torch.cuda.synchronize()
            a = time.perf_counter()
            dt.dt_count(h, d, d, d)
            ts.append((time.perf_counter() - a) * 1e3)
        pk = dt.dt_ctx_last_profile(ctx)
        print(json.dumps({"quick": True, "ms_per_step": round(ms_step, 3), "value": round(value, 1),
                          "count_ms": round(statistics.median(ts[1:]), 4),
                          "kernel_ms_step": {k: round(float(np.mean([p[k] for p in prof])), 4) for k in prof[0]},
                          "kernel_ms_count": {k: round(float(v), 4) for k, v in pk.items() if v > 0},
                          "count_roofline": count_roofline(st, statistics.median(ts[1:]),
                                                           {k: round(float(pk[k]), 4) for k in (
                                                               "unit", "light", "medium", "heavy_prefix",
                                                               "heavy_count", "reduce")}),
                          "build_ms": {"peel": round(st["ms_peel"], 3), "orient": round(st["ms_orient"], 3),
                                       "triangles": round(st["ms_triangles"], 3),
                                       "schedule": round(st["ms_schedule"], 3)},
                          "stats": {k: v for k, v in st.items() if isinstance(v, int)}}), flush=True)
        dt.dt_graph_free(h)
        dt.dt_ctx_destroy(ctx)
        torch.cuda.synchronize()
        torch.cuda.empty_cache()
        return

    # the one-shot path: ordering, orientation and enumeration that counts as it goes (no stored
    # triangle list); it drops the build, which is made again afterwards
    ts = []
    for _ in range(args.steps + 1):
        torch.cuda.synchronize()
        a = time.perf_counter()
        o1 = dt.dt_count_oneshot(h, d, d, d)
        ts.append((time.perf_counter() - a) * 1e3)
    p1 = dt.dt_ctx_last_profile(ctx)
    oneshot = {"ms": round(statistics.median(ts[1:]), 3),
               "edges_per_s": round(g.m / (statistics.median(ts[1:]) / 1e3), 1),
               "fused_enumerate_count_ms": round(p1["tri_fill"], 3),
               "matches_step": bool((o1 == out).all())}
    log("oneshot", oneshot)
    dt.dt_graph_build(h)
    st0 = dt.dt_graph_stats(h)

    # count alone on the resident build, per delta up to infinity (Section 6: the time should not
    # depend on the deltas), with the instrumented count's visits against Theorem 1's bound
    count_ms, visits, count_kernels_by_delta = {}, {}, {}
    sweep_ds = (600, 3600, 86400, 10**6, dt.DT_INF)
    for dd in sweep_ds:
        name = "inf" if dd == dt.DT_INF else str(dd)
        ts = []
        for _ in range(7 if dd != d else 21):
            torch.cuda.synchronize()
            a = time.perf_counter()
            dt.dt_count(h, dd, dd, dd)
            ts.append((time.perf_counter() - a) * 1e3)
        count_ms[name] = round(statistics.median(ts[1:]), 4)
        pk = dt.dt_ctx_last_profile(ctx)
        count_kernels_by_delta[name] = {k: round(float(pk[k]), 4) for k in
                                        ("unit", "light", "medium", "heavy_prefix", "heavy_count") if pk[k] > 0}
        got_v, v = dt.dt_count_visits(h, dd, dd, dd)
        visits[name] = int(v)
        if dd == dt.DT_INF:
            inf_identity = int(got_v.sum()) == st0["sum_sigma3"]
    bound = 2 * 48 * st0["degeneracy"] * g.m
    cm = list(count_ms.values())
    flat = {"count_ms": count_ms, "max_over_min": round(max(cm) / min(cm), 3),
            "visits": visits, "visit_bound": bound, "visits_within_bound": max(visits.values()) <= bound,
            "inf_sum_equals_sum_sigma3": inf_identity, "kernel_ms": count_kernels_by_delta}
    log("count ms", flat)

    # a delta sweep (eight triples, the shape of the paper's parameter sweeps) in one pass against
    # eight separate counts
    sweep_d = [(x, x, x) for x in (60, 600, 1800, 3600, 7200, 21600, 86400, 604800)]
    ref_sweep = np.array([dt.dt_count(h, *x) for x in sweep_d])
    ts_one, ts_sep = [], []
    for _ in range(11):
        torch.cuda.synchronize()
        a = time.perf_counter()
        got_sweep = dt.dt_count_sweep(h, sweep_d)
        ts_one.append((time.perf_counter() - a) * 1e3)
        a = time.perf_counter()
        for x in sweep_d:
            dt.dt_count(h, *x)
        ts_sep.append((time.perf_counter() - a) * 1e3)
    sweep = {"deltas": [x[0] for x in sweep_d], "one_pass_ms": round(statistics.median(ts_one[1:]), 4),
             "separate_ms": round(statistics.median(ts_sep[1:]), 4),
             "matches_separate": bool((got_sweep == ref_sweep).all())}
    sweep["speedup"] = round(sweep["separate_ms"] / sweep["one_pass_ms"], 2)
    log("sweep", sweep)

    # roofline of the dominant kernel of the step (event-timed on the library's stream)
    mean = {k: float(np.mean([p[k] for p in prof])) for k in prof[0]}
    heavy_bytes = st["alg_bytes"] - st["alg_bytes_light"] - st["alg_bytes_medium"] - st["alg_bytes_unit"]
    alg = {
        "peel": st["alg_bytes_peel"],
        "peel_adj": 0,
        "peel_tail": 0,
        "core": st["alg_bytes_peel"],
        "relayout": 25 * st["m_loaded"],
        "tri_count": 4 * (st["m_static"] + st["tri_candidates"]),
        "tri_fill": 4 * (st["m_static"] + st["tri_candidates"]) + 12 * st["n_static_triangles"],
        "light": st["alg_bytes_light"],
        "medium": st["alg_bytes_medium"],
        "unit": st["alg_bytes_unit"],
        "heavy_prefix": heavy_bytes,
        "heavy_count": heavy_bytes,
        "reduce": 64,
    }
    dom = max(mean, key=lambda k: mean[k])
    achieved = alg[dom] / (mean[dom] / 1e3) / 1e9 if mean[dom] > 0 else 0.0
    roofline = {"bound": "hbm", "kernel": dom, "achieved": round(achieved, 2),
                "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 5),
                "traffic": measured_traffic(dom), "alg_bytes": int(alg[dom]),
                "avg_ms": round(mean[dom], 4)}
    # the same figures for every build kernel of a millisecond or more (the peel's grid kernel and
    # the enumeration take within a few percent of the same time)
    roofline_by_kernel = {}
    for k in sorted(mean, key=lambda k: -mean[k]):
        if mean[k] >= 1.0 and alg.get(k):
            a = alg[k] / (mean[k] / 1e3) / 1e9
            roofline_by_kernel[k] = {"avg_ms": round(mean[k], 4), "alg_bytes": int(alg[k]),
                                     "achieved": round(a, 2), "frac": round(a / HBM_PEAK_GBS, 5),
                                     "traffic": measured_traffic(k)}
    count_kernels = {k: round(mean[k], 4) for k in ("unit", "light", "medium", "heavy_prefix",
                                                     "heavy_count", "reduce")}

    cpu = cpu_dottt = None
    parity = {}
    if not args.no_cpu:
        import oracle
        threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
        # whole-span parity of the full graph at every delta of its sweep (Definition 1 against the
        # oracle, outside the timed region); the run at the headline delta is the CPU baseline
        for dd in (600, 3600, 86400):
            a = time.perf_counter()
            want = oracle.count(g.n, g.src, g.dst, g.t, dd, dd, dd, nthreads=threads)
            cpu_s = time.perf_counter() - a
            got = dt.dt_count(h, dd, dd, dd)
            parity[str(dd)] = {"gpu_matches_oracle": bool((got == want).all()), "oracle_s": round(cpu_s, 3),
                               "counts": got.tolist()}
            log("whole-span parity", dd, parity[str(dd)])
            if dd == d:
                cpu = {"value": round(g.m / cpu_s, 1), "unit": "temporal edges/s", "cores": threads,
                       "kind": "oracle", "seconds": round(cpu_s, 3),
                       "sample": f"the whole graph ({g.m} edges), deltas ({d},{d},{d})",
                       "gpu_matches_oracle": parity[str(dd)]["gpu_matches_oracle"]}
        # the paper's own algorithm, sequential (its setting), on a sample
        lo = int(g.t.min())
        hi2 = lo + int((int(g.t.max()) - lo) * args.cpu_dottt_frac)
        keep2 = (g.t >= lo) & (g.t <= hi2)
        a = time.perf_counter()
        want2, core_s = oracle.cpu_dottt(g.n, g.src, g.dst, g.t, d, d, d, lo, hi2, seconds=True)
        dottt_s = time.perf_counter() - a
        got2 = dt.dt_count(h, d, d, d, lo, hi2)
        cpu_dottt = {"value": round(int(keep2.sum()) / dottt_s, 1), "unit": "temporal edges/s", "cores": 1,
                     "kind": "cpu_dottt", "seconds": round(dottt_s, 3),
                     "seconds_after_extraction": round(core_s, 3),
                     "sample": f"edges with t in the first {args.cpu_dottt_frac:g} of the span "
                               f"({int(keep2.sum())} of {g.m} edges), deltas ({d},{d},{d})",
                     "gpu_matches": bool((got2 == want2).all())}
        log("cpu dottt", cpu_dottt)

    medium = None
    if args.medium and args.workload == "full":
        medium = run_medium(dt, ctx, d, not args.no_cpu)

    # the autotuner on this graph (outside the timed region): its choice, the time it takes, and
    # the count under the schedule it picks; then back to the defaults
    a = time.perf_counter()
    dt.dt_graph_set_tuning(h, autotune=2)
    tune_s = time.perf_counter() - a
    stt = dt.dt_graph_stats(h)
    ts = []
    for _ in range(11):
        torch.cuda.synchronize()
        a = time.perf_counter()
        got_t = dt.dt_count(h, d, d, d)
        ts.append((time.perf_counter() - a) * 1e3)
    autotuner = {"autotuned": stt["autotuned"], "light_pair_cap": stt["light_pair_cap_used"],
                 "medium_cost_pct": stt["medium_cost_pct_used"],
                 "light_blocks_per_cu": stt["light_blocks_per_cu"],
                 "medium_blocks_per_cu": stt["medium_blocks_per_cu"], "tuning_s": round(tune_s, 2),
                 "count_ms_tuned": round(statistics.median(ts[1:]), 4),
                 "count_ms_default": count_ms[str(d)], "counts_equal": bool((got_t == out).all())}
    log("autotuner", autotuner)
    dt.dt_graph_set_tuning(h, autotune=1)

    batched = served = None
    if args.batch_graphs > 0:
        batched, bgraphs = run_batched(dt, ctx, args.batch_graphs, not args.no_cpu)
        served = run_served(dt, ctx, [(h, g.n, int(g.t.min()), int(g.t.max()))] + bgraphs[:64],
                            args.serve_seconds, args.serve_warmup, args.serve_rate)
        for bh, *_ in bgraphs:
            dt.dt_graph_free(bh)

    line = {
        "metric": "temporal edges/s counted (63M-edge graph, delta=3600s); p50/p99 query latency",
        "value": round(value, 1),
        "unit": "temporal edges/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(ms_step, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "int64", "data": "synthetic",
        "config": {"workload": g.name, "n": g.n, "m": g.m, "deltas": [d, d, d],
                   "step": "peel + orient + triangles + schedule + count + reduce",
                   "parallelism": "single GPU"},
        "counts": out.tolist(),
        "count_ms": count_ms,
        "delta_independence": flat,
        "count_edges_per_s": round(g.m / (count_ms[str(d)] / 1e3), 1),
        "sweep": sweep,
        "oneshot": oneshot,
        "kernel_ms": {k: round(v, 4) for k, v in mean.items()},
        "split": {"light_pair_cap": st["light_pair_cap_used"], "medium_cost_pct": st["medium_cost_pct_used"],
                  "light_blocks_per_cu": st["light_blocks_per_cu"],
                  "medium_blocks_per_cu": st["medium_blocks_per_cu"]},
        "autotuner": autotuner,
        "build_ms": {"peel": round(st["ms_peel"], 3), "orient": round(st["ms_orient"], 3),
                     "triangles": round(st["ms_triangles"], 3),
                     "schedule": round(st["ms_schedule"], 3)},
        "graph": {"m_static": st["m_static"], "static_triangles": st["n_static_triangles"],
                  "degeneracy": st["degeneracy"], "max_multiplicity": st["max_multiplicity"],
                  "unit": st["n_unit_triangles"],
                  "light": st["n_light_triangles"], "medium": st["n_medium_triangles"],
                  "heavy": st["n_heavy_triangles"], "heavy_slots": st["heavy_slots"],
                  "contested": st["n_contested_triangles"],
                  "tri_candidates": st["tri_candidates"],
                  "alg_bytes_count": st["alg_bytes"]},
        "roofline": roofline,
        "roofline_by_kernel": roofline_by_kernel,
        "count_roofline": count_roofline(st, count_ms[str(d)], count_kernels),
        "cpu_baseline": cpu,
        "parity_whole_span": parity,
        "medium": medium,
        "cpu_dottt": cpu_dottt,
        "batched": batched,
        "served": served,
    }
    dt.dt_graph_free(h)
    dt.dt_ctx_destroy(ctx)
    # nothing of ours or torch's left on the device before the interpreter's teardown
    torch.cuda.synchronize()
    torch.cuda.empty_cache()
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
