#!/usr/bin/env python3
"""Benchmark of the sliding super point hot path on one MI355X.

Workload (single router at scale): 2^26 synthetic packets over 60 time slices, window 10,
threshold 1024; SRE array 11 x 16384 x 8 u16, SLE array 5 x 65536 x 1024 u16.  One step is
the whole job: reset the sketch, ingest each slice's packets (per-packet SRE + SLE stamp
writes), and after every slice with a full window scan it (row live counts + hot SREs,
candidate recovery, union-SLE estimates, filter, ordered report) -- 60 ingests, 51 scans.
All packets are resident in device memory before the timed region starts.

Prints ONE JSON line.  `value` is whole-job packets per second (ingest and scans both
inside the timed region).  Per-kernel durations come from HIP events the library records
on the stream each kernel runs on, inside the timed region.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0
# 256 CUs x 64 lanes x 2.4 GHz: one 32-bit integer VALU operation per lane per clock
PEAK_INT32_TOPS = 256 * 64 * 2.4e9 / 1e12
JOIN_OPS_PER_TEST = 4
# one wave64 VALU instruction per CU per clock (four SIMD16 units, four clocks each)
PEAK_VALU_WAVE_INSTR = 256 * 2.4e9
TIMED_EVERY = 4  # slices of a timed step whose dominant-kernel launches carry HIP events
METRIC = "packets/s ingested (SRE+SLE) + scan ms/slice; p99 latency; learned vs LC rel. error"


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for f in sorted(os.listdir(os.path.join(ROOT, "paper_1805_09246_amd", "csrc"))):
        with open(os.path.join(ROOT, "paper_1805_09246_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def stored_counter(kernel: str, counter: str):
    """Mean per dispatch of a rocprofv3 counter from the committed counter summary, if it was
    taken on the current kernel sources."""
    path = os.path.join(ROOT, "profiles", "counters.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        t = json.load(f)
    e = t.get(kernel)
    if not e or e.get("source_hash") != kernel_source_hash():
        return None
    return e.get("counters", {}).get(counter)


def stored_traffic(kernel: str):
    """HBM bytes per launch from the committed rocprofv3 counter summary, if it was taken on
    the current kernel sources."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        t = json.load(f)
    e = t.get(kernel)
    if not e or e.get("source_hash") != kernel_source_hash():
        return None
    return e.get("bytes_per_launch")


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(stream, params, window, threshold, n_slices_sample=10, n_scans=10,
                 tuple_growing=False):
    """The oracle timed on the host on a bounded sample: the ingest of the first slices on
    one thread and with its rows split over all threads, then a few scans (exhaustive
    candidate search over all threads), and, when asked (it takes about half a minute), the
    paper's tuple growing (Alg. 4-5, one thread) for one scan; the whole job's packets/s from
    the all-thread ingest and the exhaustive scans."""
    import numpy as np
    import oracle
    threads = oracle.default_threads()
    one, many = oracle.OracleSketch(params), oracle.OracleSketch(params)
    t_one = t_many = 0.0
    t_scan = []
    n_pk = 0
    for s in range(1, n_slices_sample + n_scans):
        p = stream.slice_pkts(s)
        t0 = time.perf_counter()
        one.ingest(p, s)
        t_one += time.perf_counter() - t0
        t0 = time.perf_counter()
        many.ingest_threads(p, s, threads)
        t_many += time.perf_counter() - t0
        n_pk += p.shape[0]
        if s >= n_slices_sample:
            t0 = time.perf_counter()
            many.scan(window, threshold, threads=threads)
            t_scan.append(time.perf_counter() - t0)
    assert np.array_equal(one.slea(), many.slea()) and np.array_equal(one.sre(), many.sre())
    base = many
    t_tuples = None
    if tuple_growing:
        t1 = time.perf_counter()
        hot = base.hot(window)
        cands = np.sort(base.join_tuples(hot, tuple_cap=1 << 25))
        base.estimate_filter(window, threshold, cands)
        t_tuples = time.perf_counter() - t1
    per_pkt = t_many / n_pk
    scan_s = sum(t_scan) / len(t_scan)
    rec = stream.recipe
    n_scans_job = rec.n_slices - window + 1
    job_s = per_pkt * rec.n_packets + scan_s * n_scans_job
    return {
        "value": rec.n_packets / job_s,
        "unit": "packets/s",
        "cores": threads,
        "cpu_model": cpu_model(),
        "hardware_threads": os.cpu_count(),
        "kind": "oracle",
        "sample": (f"oracle ingest of slices 1..{n_slices_sample + n_scans - 1} ({n_pk} packets) "
                   f"with its rows split over {threads} threads ({t_many:.2f} s; one thread "
                   f"{t_one:.2f} s) and {n_scans} scans (exhaustive candidate search on "
                   f"{threads} threads, {scan_s:.2f} s each), scaled to {rec.n_packets} packets "
                   f"and {n_scans_job} scans"),
        "ingest_pkts_per_s": 1.0 / per_pkt,
        "ingest_pkts_per_s_one_thread": n_pk / t_one,
        "scan_ms_per_slice": scan_s * 1e3,
        "scan_tuple_growing_ms_one_scan": None if t_tuples is None else t_tuples * 1e3,
    }


def detection_summary(card, k, theta, reported):
    """Def. 5 rates of the reported host lists {cur: hosts} against the exact truth, averaged
    over the scans (the paper plots them per sliding window, Figs 6-8)."""
    import numpy as np
    from oracle import truth
    rows = []
    for cur, hosts in sorted(reported.items()):
        th, _ = truth.sliding_super_points(card, k, cur, theta)
        fpr, fnr, tfr = truth.detection_rates(th, hosts)
        rows.append((len(th), len(hosts), fpr, fnr, tfr))
    a = np.asarray(rows, dtype=np.float64)
    return {"window": k, "threshold": theta, "scans": len(rows),
            "true_super_points_mean": float(a[:, 0].mean()),
            "reported_mean": float(a[:, 1].mean()),
            "FPR": float(a[:, 2].mean()), "FNR": float(a[:, 3].mean()),
            "TFR": float(a[:, 4].mean()), "TFR_max": float(a[:, 4].max())}


def accuracy_study(st, params, windows=(1, 5, 10, 20), thetas=(512, 1024, 2048)):
    """FPR / FNR / TFR (Def. 5) of the whole config-2 stream for several windows and
    thresholds: one sketch per threshold (theta fixes the sampling depth at creation), a scan
    after every slice whose window is full, exact truth from the oracle's all-windows
    distinct counts."""
    import numpy as np
    import torch
    from oracle import truth
    from paper_1805_09246_amd import sps
    t0 = time.perf_counter()
    card = truth.sliding_cardinalities(st, list(windows), min(thetas))
    log(f"exact truth for windows {list(windows)} in {time.perf_counter() - t0:.1f} s")
    pk = torch.from_numpy(st.pkts.view(np.int32)).cuda()
    offs = [int(v) for v in st.slice_off]
    n_sl = st.recipe.n_slices
    table = []
    for theta in thetas:
        # long windows at low thresholds recover more candidates than the default capacity
        g = sps.Sketch(dict(params, theta=theta, cand_cap=1 << 22))
        rep = {k: {} for k in windows}
        over = {k: 0 for k in windows}  # scans whose candidates overflowed the capacity
        for s in range(1, n_sl + 1):
            g.ingest(pk[offs[s - 1]:offs[s]], s)
            for k in windows:
                if s >= k:
                    try:
                        rep[k][s] = g.scan(k, float(theta))["host"]
                    except sps.SpsError as e:
                        if e.code != sps.SPS_ECAPACITY:
                            raise
                        over[k] += 1  # the SRE array is saturated at this window
        g.close()
        for k in windows:
            row = detection_summary(card, k, theta, rep[k]) if rep[k] else \
                {"window": k, "threshold": theta, "scans": 0}
            row["scans_saturated"] = over[k]
            table.append(row)
            log(f"theta {theta} window {k}: " + json.dumps(table[-1]))
    return table


def discrete_extra(slices, params, window, threshold, log_fn):
    """The discrete variant (one bit per recorder, set by 32-bit atomic or: RE and LE of
    Sec. 3.2 and Sec. 4) on the config-2 stream: the time axis cut into discrete windows of
    `window` slices; each window starts from a reset sketch, ingests its slices and ends with
    a scan."""
    import numpy as np
    import torch
    from paper_1805_09246_amd import sps
    g = sps.Sketch(dict(params, mode=sps.MODE_DISCRETE))
    n_sl = len(slices)

    def run():
        kept = []
        for w0 in range(0, n_sl - window + 1, window):
            g.reset()
            for s in range(w0 + 1, w0 + window + 1):
                sps.sps_ingest(g.h, slices[s - 1], s)
            kept.append(len(g.scan(1, threshold)))
        return kept

    run()
    torch.cuda.synchronize()
    sps.sps_profile_enable(True, stages={"ingest", "scan", "fill"})
    sps.sps_profile_read()
    t0 = time.perf_counter()
    kept = run()
    wall = time.perf_counter() - t0
    prof = sps.sps_profile_read()
    sps.sps_profile_enable(False)
    n_pk = sum(int(x.shape[0]) for x in slices[:len(kept) * window])
    out = {
        "workload": f"config-2 stream in discrete windows of {window} slices, bit recorders",
        "sketch_MiB": g.nbytes / 2 ** 20,
        "ingest_pkts_per_s": n_pk / (prof["ingest"][0] / 1e3),
        "ingest_us_per_slice": 1e3 * prof["ingest"][0] / prof["ingest"][1],
        "scan_ms": prof["scan"][0] / prof["scan"][1],
        "reset_us": 1e3 * prof["fill"][0] / max(1, prof["fill"][1]),
        "windows": len(kept), "hosts_reported": kept, "wall_s": wall,
    }
    g.close()
    return out


def merge_extra(log_fn):
    """Config 3: 16 routers with lognormal traffic, one captured graph per slice (batched
    ingest of every router's slice, then max-merge into the global sketch and its scan)."""
    import numpy as np
    import torch
    from paper_1805_09246_amd import sps
    from synth import make_multi_stream
    from synth.configs import C3_PARAMS, C3_RECIPE, C3_THRESHOLD, C3_WINDOW
    t0 = time.perf_counter()
    rs = make_multi_stream(C3_RECIPE)
    log_fn(f"config-3 streams generated in {time.perf_counter() - t0:.1f} s")
    pk = [torch.from_numpy(r.pkts.view(np.int32)).cuda() for r in rs]
    offs = [[int(v) for v in r.slice_off] for r in rs]
    n_total = sum(r.pkts.shape[0] for r in rs)
    routers = [sps.Sketch(C3_PARAMS) for _ in rs]
    merged = sps.Sketch(C3_PARAMS)
    n_sl = C3_RECIPE.n_slices
    cap = 8192
    res = torch.zeros((n_sl, cap * 24), dtype=torch.uint8, device="cuda")
    info = torch.zeros((n_sl, 8), dtype=torch.int32, device="cuda")
    st = torch.cuda.Stream()  # a capturable stream (not the legacy default stream)
    torch.cuda.synchronize()

    def slice_pk(s):
        return [pk[j][offs[j][s - 1]:offs[j][s]] for j in range(len(rs))]

    # the autotuner picks the batched launch shape on slice 1 (ingesting it)
    best, _ = sps.sps_autotune_ingest([r.h for r in routers], slice_pk(1), 1, st)
    for r in routers:
        sps.sps_set_tuning(r.h, **best)
    torch.cuda.synchronize()
    sps.sps_profile_enable(True, stages={"ingest_batched", "merge", "scan"})
    sps.sps_profile_read()
    t0 = time.perf_counter()
    for s in range(2, n_sl + 1):
        sps.sps_graph_begin(st)
        try:
            sps.sps_ingest_batched([r.h for r in routers], slice_pk(s), s, st)
            if s >= C3_WINDOW:
                merged.merge(routers, st)
                sps.sps_scan_async(merged.h, C3_WINDOW, C3_THRESHOLD, res[s - 1], cap,
                                   info[s - 1], st)
        finally:
            g = sps.sps_graph_end(st)
        sps.sps_graph_launch(g, st)
        st.synchronize()
        sps.sps_graph_destroy(g)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    prof = sps.sps_profile_read()
    sps.sps_profile_enable(False)
    # graph launches are not bracketed; time each stage once more, eagerly, on the last state
    sps.sps_profile_enable(True, stages={"ingest_batched", "merge", "scan"})
    sps.sps_profile_read()
    sps.sps_ingest_batched([r.h for r in routers], slice_pk(n_sl), n_sl, st)
    merged.merge(routers, st)
    sps.sps_scan_async(merged.h, C3_WINDOW, C3_THRESHOLD, res[n_sl - 1], cap, info[n_sl - 1], st)
    st.synchronize()
    prof = sps.sps_profile_read()
    sps.sps_profile_enable(False)
    inf = info.cpu().numpy()
    tau, _, row_len = merged.derived()
    p = C3_PARAMS
    state = 2 * ((p["r"] << p["q"]) * p["eta"] + p["rp"] * row_len)
    merge_ms = prof["merge"][0]
    merge_bytes = (len(routers) + 2) * state
    pk_last = sum(x.shape[0] for x in slice_pk(n_sl))
    out = {
        "workload": f"{len(rs)} routers, lognormal sizes (median 2^22, sigma 1), {n_sl} slices, "
                    f"window {C3_WINDOW}, threshold {C3_THRESHOLD:.0f}, SRE {p['r']}x{1 << p['q']}x8, "
                    f"SLE {p['rp']}x{1 << p['qp']}x{p['etap']}",
        "packets": int(n_total),
        "graph_per_slice_packets_per_s": sum(sum(x.shape[0] for x in slice_pk(s))
                                             for s in range(2, n_sl + 1)) / wall,
        "batched_tuning": best,
        "batched_ingest_pkts_per_s": pk_last / (prof["ingest_batched"][0] / 1e3),
        "merge_ms": merge_ms,
        "merge_alg_GBps": merge_bytes / (merge_ms / 1e3) / 1e9,
        "merge_frac_of_8TBps": merge_bytes / (merge_ms / 1e3) / 1e9 / PEAK_HBM_GBS,
        "scan_ms": prof["scan"][0],
        "hosts_reported_last_scan": int(inf[n_sl - 1, 0]),
        "candidates_last_scan": int(inf[n_sl - 1, 1]),
    }
    for r in routers:
        r.close()
    merged.close()
    del pk
    return out


def serving_extra(pool, log_fn, runs=3):
    """Config 4: the serving loop in real time.  Latency of a batch: its arrival to the
    completion of the slice that ingested it (the host clock stored by a notification the
    stream runs right after the slice's graph), and to its report (results copied back).  Three consecutive runs of
    120 slices on the same resident routers, each with its own arrival schedule; the batched
    ingest's launch shape is autotuned first on a sample of batches."""
    import numpy as np
    import torch
    from paper_1805_09246_amd.serve import Server, poisson_schedule, run_simulation
    from synth.configs import (C4_BUDGET, C4_PARAMS, C4_RATE, C4_ROUTERS, C4_SEED, C4_SLICE_S,
                               C4_SLICES, C4_THRESHOLD, C4_WINDOW)
    srv = Server(C4_PARAMS, C4_WINDOW, C4_THRESHOLD, C4_BUDGET)
    for r in range(C4_ROUTERS):
        srv.admit(r)
    # one slice's worth of batches of the serving process, for the tuner
    t, rt, sz = poisson_schedule(C4_SEED ^ 0x7E57, C4_RATE, C4_SLICE_S, C4_ROUTERS)
    offs = np.random.Generator(np.random.Philox(7)).integers(0, pool.shape[0] - sz.max(), len(sz))
    tune, _ = srv.autotune([(int(r), pool[int(o):int(o) + int(n)])
                            for r, o, n in zip(rt, offs, sz)])
    log_fn(f"serving: batched ingest tuned to {tune}")
    per_run = []
    n_pk_all, wall_all = 0, 0.0
    for run in range(runs):
        first = len(srv.reports)
        sched = poisson_schedule(C4_SEED + run, C4_RATE, C4_SLICES * C4_SLICE_S, C4_ROUTERS)
        wall, n_pk = run_simulation(srv, pool, sched, C4_SLICE_S, C4_SLICES, seed=1 + run)
        reps = srv.reports[first:]
        lat = np.array([x for r in reps for x in r.latencies])
        rlat = np.array([x for r in reps for x in r.report_latencies])
        per_run.append({"p50_ms": float(np.percentile(lat, 50) * 1e3),
                        "p99_ms": float(np.percentile(lat, 99) * 1e3),
                        "max_ms": float(lat.max() * 1e3),
                        "report_p50_ms": float(np.percentile(rlat, 50) * 1e3),
                        "report_p99_ms": float(np.percentile(rlat, 99) * 1e3),
                        "batches": int(len(lat)), "packets_per_s": n_pk / wall})
        n_pk_all += n_pk
        wall_all += wall
        log_fn(f"serving run {run}: {len(lat)} batches, {n_pk} packets in {wall:.2f} s, "
               f"p50 {per_run[-1]['p50_ms']:.2f} ms, p99 {per_run[-1]['p99_ms']:.2f} ms")
    hm = {k: (float(np.mean(v)), len(v)) for k, v in srv.host_ms.items() if v}
    p99 = [r["p99_ms"] for r in per_run]
    p50 = [r["p50_ms"] for r in per_run]
    out = {
        "workload": f"{C4_ROUTERS} routers, Poisson batches 4Ki-4Mi at {C4_RATE:.0e} pkt/s, "
                    f"{runs} runs of {C4_SLICES} slices of {C4_SLICE_S * 1e3:.0f} ms, "
                    f"window {C4_WINDOW}",
        "packets_per_s": n_pk_all / wall_all,
        "offered_packets_per_s": C4_RATE,
        "p50_latency_ms": float(np.median(p50)),
        "p99_latency_ms": float(np.median(p99)),
        "p99_latency_ms_range": [min(p99), max(p99)],
        "p50_latency_ms_range": [min(p50), max(p50)],
        "latency": "batch arrival to completion of its slice on the GPU (median over runs)",
        "runs": per_run,
        "batched_tuning": tune,
        "host_ms_per_slice": {k: {"mean_ms": v[0], "slices": v[1]} for k, v in hm.items()},
        "resident_sketches": len(srv.slots),
        "resident_GiB": srv.used_bytes() / 2 ** 30,
        "incomplete_reports": srv.incomplete,
    }
    srv.close()
    torch.cuda.synchronize()
    return out


def learned_extra(log_fn):
    """Config 5: train the estimator on generated hosts; held-out error vs linear counting."""
    import numpy as np
    from paper_1805_09246_amd import learned
    from synth.configs import C5_PARAMS, C5_SEEDS, C5_TEST, C5_TRAIN, C5_VAL
    t0 = time.perf_counter()
    bases = learned.make_backgrounds(C5_PARAMS, C5_SEEDS[0])
    tr = learned.generate(C5_PARAMS, C5_TRAIN, C5_SEEDS[0], bases=bases, log=log_fn)
    va = learned.generate(C5_PARAMS, C5_VAL, C5_SEEDS[1], bases=bases)
    te = learned.generate(C5_PARAMS, C5_TEST, C5_SEEDS[2], bases=bases)
    # held-out hosts under another arrival law: fresh peers spread evenly over the window
    ood = learned.generate(C5_PARAMS, C5_TEST, C5_SEEDS[2] ^ 0x0D, bases=bases, law=1)
    for b in bases:
        b.close()
    t_gen = time.perf_counter() - t0
    t0 = time.perf_counter()
    w = learned.train(tr, epochs=20, batch=4096, lr=3e-3, log=log_fn)
    import torch
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t0
    gate = learned.fit_gate(tr, va, learned.predict(w, va))
    est, use = learned.gated(te, learned.predict(w, te), gate)
    e_lc = np.abs(te.lc - te.cards) / te.cards
    e_ml = np.abs(est - te.cards) / te.cards
    o_est, o_use = learned.gated(ood, learned.predict(w, ood), gate)
    o_lc = np.abs(ood.lc - ood.cards) / ood.cards
    o_ml = np.abs(o_est - ood.cards) / ood.cards
    return {
        "workload": f"{C5_TRAIN} training / {C5_VAL} validation / {C5_TEST} held-out hosts, "
                    "cardinality log-uniform 1..1e6, window 10",
        "lc_mean_rel_err": float(e_lc.mean()),
        "mlp_mean_rel_err": float(e_ml.mean()),
        "mlp_used_frac": float(use.mean()),
        "gate_min_live": int(gate.min_live),
        "per_decade": [dict(d, mlp=m["mean_rel_err"]) for d, m in
                       zip(learned.rel_err_table(te.cards, te.lc),
                           learned.rel_err_table(te.cards, est))],
        "even_arrivals": {
            "hosts": int(len(ood.cards)),
            "lc_mean_rel_err": float(o_lc.mean()), "mlp_mean_rel_err": float(o_ml.mean()),
            "mlp_used_frac": float(o_use.mean()),
            "per_decade": [dict(d, mlp=m["mean_rel_err"]) for d, m in
                           zip(learned.rel_err_table(ood.cards, ood.lc),
                               learned.rel_err_table(ood.cards, o_est))]},
        "dataset_s": t_gen,
        "train_s": t_train,
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-probes", action="store_true")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the merge (config 3), serving (config 4) and learned-estimator "
                         "(config 5) legs")
    ap.add_argument("--scan-overlap", type=int, default=0, choices=(0, 1, 2),
                    help="1: row-count sweep in waves of its own inside the candidate search's "
                         "launch; 2: the sweep as a kernel of its own after the search; 0: the "
                         "library's default")
    ap.add_argument("--tuning-cache", default="", metavar="JSON",
                    help="ingest launch shape from this tuning cache file when it holds the "
                         "workload's shape; otherwise autotune and write the file")
    ap.add_argument("--cpu-tuple-growing", action="store_true",
                    help="also time the oracle's tuple-growing candidate search (Alg. 4-5) for "
                         "one scan in the CPU baseline (about half a minute on 16 cores)")
    ap.add_argument("--no-discrete", action="store_true",
                    help="skip the discrete-window (bit recorder) leg")
    ap.add_argument("--no-accuracy", action="store_true",
                    help="skip the detection rates of the timed step's reports")
    ap.add_argument("--accuracy-study", action="store_true",
                    help="only print the FPR/FNR/TFR table over windows 1, 5, 10, 20 and "
                         "thresholds 512, 1024, 2048 on the config-2 stream")
    ap.add_argument("--merge-only", action="store_true",
                    help="only run the config-3 leg (16 routers, batched ingest, merge, scan of "
                         "the merged sketch) and print its JSON (for profiling its kernels)")
    ap.add_argument("--copy-probe", type=int, default=0, metavar="MIB",
                    help="only run one plain device copy of MIB MiB (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported (the "
              f"sharded design is described in DESIGN.md)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_1805_09246_amd import sps
    from synth import make_stream
    from synth.configs import C2_PARAMS, C2_RECIPE, C2_THRESHOLD, C2_WINDOW

    torch.cuda.set_device(0)
    if args.copy_probe:
        a = torch.ones(args.copy_probe << 20, dtype=torch.uint8, device="cuda")
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_probe_bytes": a.numel()}), flush=True)
        return
    if args.merge_only:
        print(json.dumps({"distributed_merge": merge_extra(log)}), flush=True)
        return
    rec, params, K_WIN, THETA = C2_RECIPE, C2_PARAMS, C2_WINDOW, C2_THRESHOLD
    t0 = time.perf_counter()
    st = make_stream(rec)
    log(f"stream generated in {time.perf_counter() - t0:.1f} s")
    if args.accuracy_study:
        print(json.dumps({"workload": rec.name, "accuracy": accuracy_study(st, params)}),
              flush=True)
        return
    pkts = torch.from_numpy(st.pkts.view(np.int32)).cuda()
    offs = [int(v) for v in st.slice_off]
    slices = [pkts[offs[s - 1]:offs[s]] for s in range(1, rec.n_slices + 1)]
    sk = sps.Sketch(params)
    n_scans = rec.n_slices - K_WIN + 1
    cap = 8192
    res = torch.zeros((n_scans, cap * 24), dtype=torch.uint8, device="cuda")
    info = torch.zeros((n_scans, 8), dtype=torch.int32, device="cuda")

    def step(timed=None):
        """One pass of the whole path; with `timed` (stage names), the launches of those
        stages in every TIMED_EVERY-th slice carry HIP events (from their own dispatch)."""
        sk.reset()
        for s in range(1, rec.n_slices + 1):
            on = timed is not None and (s - 1) % TIMED_EVERY == 0
            if on:
                sps.sps_profile_enable(True, stages=timed)
            sps.sps_ingest(sk.h, slices[s - 1], s)
            if s >= K_WIN:
                j = s - K_WIN
                sps.sps_scan_async(sk.h, K_WIN, THETA, res[j], cap, info[j])
            if on:
                sps.sps_profile_enable(False)

    # launch shape of the ingest: from the tuning cache file when it holds this shape, else
    # autotuned on slice 1 (re-ingesting it is idempotent and every step starts from a reset)
    tuning = None
    if args.tuning_cache and os.path.exists(args.tuning_cache):
        sps.sps_tuning_cache_load(args.tuning_cache)
        tuning = sps.sps_tuning_lookup(params, False)
        if tuning is not None:
            sps.sps_set_tuning(sk.h, **tuning)
    if tuning is None:
        tuning, _ = sps.sps_autotune_ingest([sk.h], [slices[0]], 1)
        if args.tuning_cache:
            sps.sps_tuning_cache_save(args.tuning_cache)
    log(f"ingest tuned to {tuning}")
    if args.scan_overlap:
        sps.sps_set_tuning(sk.h, scan_overlap=args.scan_overlap)
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    inf = info.cpu().numpy()
    if (inf[:, sps.INFO_FLAGS] != 0).any():
        raise RuntimeError("scan buffers overflowed")
    log(f"warm-up done; hosts reported per scan: {int(inf[:, 0].min())}..{int(inf[:, 0].max())}")
    # one profiled step with every kernel timed by its own dispatch (HIP events attached to
    # the launch: no packets added to the stream): the breakdown and the dominant kernel; then
    # one step with every whole scan bracketed by a pair of recorded events
    kernel_stages = ("ingest", "scan_stats", "scan_rows", "join", "estimate", "sort", "fill")
    sps.sps_profile_enable(True, stages=set(kernel_stages))
    sps.sps_profile_read()
    step()
    prof_all = sps.sps_profile_read()
    sps.sps_profile_enable(True, stages={"scan"})
    step()
    prof_scan = sps.sps_profile_read()
    dominant = max(kernel_stages, key=lambda k: prof_all[k][0])
    # timed region: the dominant kernel's launches in every TIMED_EVERY-th slice carry events
    # from their own dispatch (an event-carrying launch costs a few us of stream time, so
    # timing every launch would slow the step it measures)
    sps.sps_profile_enable(False)
    sps.sps_profile_read()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step(timed={dominant})
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    prof = sps.sps_profile_read()
    log(f"timed {args.steps} steps in {elapsed:.3f} s; dominant kernel stage: {dominant}")

    # one more step with every scan bracketed by events, each followed by the copy of its
    # info words and kept results to pinned host memory: the median scan including the D2H
    h_info = torch.zeros(8, dtype=torch.int32).pin_memory()
    h_res = torch.zeros(cap * 24, dtype=torch.uint8).pin_memory()
    scan_ev = []
    sk.reset()
    for s in range(1, rec.n_slices + 1):
        sps.sps_ingest(sk.h, slices[s - 1], s)
        if s >= K_WIN:
            j = s - K_WIN
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            sps.sps_scan_async(sk.h, K_WIN, THETA, res[j], cap, info[j])
            h_info.copy_(info[j], non_blocking=True)
            h_res.copy_(res[j], non_blocking=True)
            e1.record()
            scan_ev.append((e0, e1))
    torch.cuda.synchronize()
    scan_median_ms = float(np.median([a.elapsed_time(b) for a, b in scan_ev]))

    total_pkts = args.steps * rec.n_packets
    value = total_pkts / elapsed
    tau, _, row_len = sk.derived()
    stores_per_pkt = params["rp"] + params["r"] * 2.0 ** -tau
    ingest_bytes_per_pkt = 8 + 2 * stores_per_pkt
    # the row-count sweep streams the SLE array once (inside the candidate search's launch by
    # default, else k_scan_rows); the hot-SRE pass (k_scan_sre) streams the SRE array and
    # writes the hot bitmap and the join table
    rows_bytes = 2 * params["rp"] * row_len
    n_sre = params["r"] << params["q"]
    sre_bytes = 2 * n_sre * params["eta"] + n_sre // 8 + n_sre // 8
    fused = sps.sps_get_scan_overlap(sk.h) and not prof_all["scan_rows"][1]
    # the candidate search: every expanded node tests its 2^delta extensions (Alg. 4-5), each
    # test a shift, xor, mask and bit test of 32-bit integers
    inf = info.cpu().numpy().astype(np.int64)
    nodes_per_scan = float(np.mean(inf[:, sps.INFO_NODES_LO] & 0xFFFFFFFF
                                   | (inf[:, sps.INFO_NODES_HI] << 32)))
    join_ops = nodes_per_scan * (1 << params["delta"]) * JOIN_OPS_PER_TEST
    stage_ms = {k: {"total_ms": round(v[0], 3), "launches": v[1],
                    "avg_us": round(1e3 * v[0] / v[1], 2) if v[1] else None}
                for k, v in list(prof_all.items()) + [("scan", prof_scan["scan"])] if v[1]}
    compact = (tuning or {}).get("host_classes", 8) > 1
    kernel_names = {"ingest": "k_ingest_compact" if compact else "k_ingest<false, false>",
                    "scan_stats": "k_scan_sre",
                    "scan_rows": "k_scan_rows<false>",
                    "join": "k_join<true, 1>" if fused else "k_join<true, 0>",
                    "estimate": "k_estimate", "sort": "k_rank_sort", "fill": "k_fill_zero"}

    hbm_bytes = {"ingest": rec.n_packets / rec.n_slices * ingest_bytes_per_pkt,
                 "scan_stats": sre_bytes, "scan_rows": rows_bytes}
    if fused:  # the search's launch also streams the SLE array
        hbm_bytes["join"] = rows_bytes

    def search_roofline(avg_s):
        a = join_ops / avg_s / 1e12
        out = {"bound": "alu", "achieved": round(a, 4), "peak": PEAK_INT32_TOPS,
               "unit": "Tops/s (int32 lane ops)", "frac": round(a / PEAK_INT32_TOPS, 4),
               "nodes_per_launch": int(nodes_per_scan), "alg_ops_per_launch": int(join_ops)}
        # executed work: wave-level VALU instructions per launch (rocprofv3 SQ_INSTS_VALU,
        # when taken on these kernel sources) against the issue rate of one wave64 VALU
        # instruction per CU per clock
        valu = stored_counter(kernel_names["join"], "SQ_INSTS_VALU")
        if valu:
            out["executed_valu_instr_per_launch"] = int(valu)
            out["valu_issue_frac"] = round(valu / avg_s / PEAK_VALU_WAVE_INSTR, 4)
        return out

    def kernel_roofline(stage, avg_s):
        if stage in hbm_bytes:
            b = hbm_bytes[stage]
            a = b / avg_s / 1e9
            out = {"bound": "hbm", "achieved": round(a, 2), "peak": PEAK_HBM_GBS, "unit": "GB/s",
                   "frac": round(a / PEAK_HBM_GBS, 4), "alg_bytes_per_launch": int(b)}
            if stage == "join":  # the search beside the sweep, against its own roof
                out["search"] = search_roofline(avg_s)
            return out
        if stage == "join":
            return search_roofline(avg_s)
        return None

    avg_s = prof[dominant][0] / prof[dominant][1] / 1e3
    roofline = kernel_roofline(dominant, avg_s) or {"bound": "alu", "achieved": None,
                                                     "peak": None, "unit": None, "frac": None}
    roofline.update({"traffic": stored_traffic(kernel_names[dominant]),
                     "kernel": kernel_names[dominant], "avg_launch_us": round(avg_s * 1e6, 2),
                     "timed_launches": prof[dominant][1],
                     "timed": f"every {TIMED_EVERY}th slice of the timed steps"})
    per_kernel = {}
    for k in ("ingest", "scan_stats", "scan_rows", "join"):
        if prof_all[k][1]:
            rk = kernel_roofline(k, prof_all[k][0] / prof_all[k][1] / 1e3)
            rk["avg_launch_us_profiled_step"] = round(1e3 * prof_all[k][0] / prof_all[k][1], 2)
            per_kernel[kernel_names[k]] = rk

    out = {
        "metric": METRIC,
        "value": value,
        "unit": "packets/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * elapsed / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u16",
        "data": "synthetic",
        "config": {"workload": rec.name, "packets": rec.n_packets, "slices": rec.n_slices,
                   "window": K_WIN, "threshold": THETA,
                   "sre": f"{params['r']}x{1 << params['q']}x{params['eta']} u16",
                   "sle": f"{params['rp']}x{1 << params['qp']}x{params['etap']} u16",
                   "parallelism": "1 GPU"},
        "roofline": roofline,
        "ingest_tuning": tuning,
        "scan_overlap": sps.sps_get_scan_overlap(sk.h),
        "ingest_pkts_per_s": rec.n_packets / (prof_all["ingest"][0] / 1e3),
        "scan_ms_per_slice": prof_scan["scan"][0] / prof_scan["scan"][1],
        "scan_ms_per_slice_median_with_d2h": scan_median_ms,
        "stage_ms_one_profiled_step": stage_ms,
        "per_kernel_roofline": per_kernel,
    }

    if not args.no_accuracy:
        # detection rates of the last timed step's reports (every scan of the run)
        from oracle import truth
        t0 = time.perf_counter()
        card = truth.sliding_cardinalities(st, [K_WIN], THETA)
        inf = info.cpu().numpy()
        rep = {j + K_WIN: sps.results_to_numpy(res[j], int(inf[j, sps.INFO_KEPT]))["host"]
               for j in range(n_scans)}
        out["accuracy"] = detection_summary(card, K_WIN, THETA, rep)
        log(f"accuracy against exact truth in {time.perf_counter() - t0:.1f} s")

    if not args.no_probes:
        # measured roofline of the ingest's access pattern (same array size, same stores)
        probe = torch.zeros(params["rp"] * row_len, dtype=torch.int16, device="cuda")
        ssum = torch.zeros(1, dtype=torch.int32, device="cuda")
        n_st = int(rec.n_packets / rec.n_slices * stores_per_pkt)
        for _ in range(2):
            sps.sps_probe_scatter(probe, n_st, 1, 1)
            sps.sps_probe_stream(probe, ssum)
        torch.cuda.synchronize()
        sps.sps_profile_enable(True)
        sps.sps_profile_read()
        for i in range(10):
            sps.sps_probe_scatter(probe, n_st, 100 + i, 2)
        sc = sps.sps_profile_read()["probe"]
        for i in range(10):
            sps.sps_probe_stream(probe, ssum)
        sm = sps.sps_profile_read()["probe"]
        sps.sps_profile_enable(False)
        R_s = n_st / (sc[0] / sc[1] / 1e3)
        BW_s = probe.numel() * 2 / (sm[0] / sm[1] / 1e3)
        del probe
        # the ingest's own stores replayed from a recorded cell list (same cells, same stamp,
        # same XCD per host class, no pair reads or hashing), against the ingest of the same
        # slice into the same sketch state: the replay bounds the ingest from below
        psk = sps.Sketch(params)
        s_mid = rec.n_slices // 2
        for s in range(1, s_mid + 1):
            sps.sps_ingest(psk.h, slices[s - 1], s)
        cells, coff = sps.sps_probe_replay_record(psk.h, slices[s_mid - 1])
        torch.cuda.synchronize()
        sps.sps_profile_enable(True)
        sps.sps_profile_read()
        for i in range(10):
            sps.sps_ingest(psk.h, slices[s_mid - 1], s_mid)
            sps.sps_probe_replay(psk.h, cells, coff, s_mid)
        pr = sps.sps_profile_read()
        sps.sps_profile_enable(False)
        psk.close()
        n_mid = int(slices[s_mid - 1].shape[0])
        t_ing = pr["ingest"][0] / pr["ingest"][1] / 1e3
        t_rep = pr["probe"][0] / pr["probe"][1] / 1e3
        out["roofline_measured"] = {
            "replay_slice": s_mid, "replay_pairs": n_mid, "replay_stores": int(coff[8]),
            "replay_us": t_rep * 1e6, "ingest_same_slice_us": t_ing * 1e6,
            "replay_stores_per_s": coff[8] / t_rep,
            "ingest_roofline_pkts_per_s": n_mid / t_rep,
            "ingest_frac_of_replay": t_rep / t_ing,
            "uniform_scatter_stores_per_s": R_s, "stream_GBps": BW_s / 1e9,
            "scan_rows_frac_of_stream": (rows_bytes / (prof_all["scan_rows"][0] /
                                                       prof_all["scan_rows"][1] / 1e3)) / BW_s
            if prof_all["scan_rows"][1] else None,
        }
        del cells

    if not args.no_discrete:
        t0 = time.perf_counter()
        out["discrete"] = discrete_extra(slices, params, K_WIN, THETA, log)
        log(f"discrete in {time.perf_counter() - t0:.1f} s")

    if not args.no_extras:
        for name, fn in (("distributed_merge", lambda: merge_extra(log)),
                         ("serving", lambda: serving_extra(pkts, log)),
                         ("learned_vs_lc", lambda: learned_extra(log))):
            t0 = time.perf_counter()
            try:
                out[name] = fn()
            except Exception as e:  # report, keep the main line
                out[name] = {"error": f"{type(e).__name__}: {e}"}
            log(f"{name} in {time.perf_counter() - t0:.1f} s")
        if "serving" in out and "p99_latency_ms" in out["serving"]:
            out["p99_latency_ms"] = out["serving"]["p99_latency_ms"]
        if "learned_vs_lc" in out and "mlp_mean_rel_err" in out["learned_vs_lc"]:
            out["learned_vs_lc_rel_err"] = [out["learned_vs_lc"]["mlp_mean_rel_err"],
                                            out["learned_vs_lc"]["lc_mean_rel_err"]]

    if not args.no_cpu_baseline:
        t0 = time.perf_counter()
        out["cpu_baseline"] = cpu_baseline(st, params, K_WIN, THETA,
                                           tuple_growing=args.cpu_tuple_growing)
        log(f"cpu baseline in {time.perf_counter() - t0:.1f} s")

    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
