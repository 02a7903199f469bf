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
METRIC = "packets/s ingested (SRE+SLE) + scan ms/slice; p99 latency; learned vs LC rel. error"


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for f in sorted(os.listdir(os.path.join(ROOT, "paper_1805_09246_amd", "csrc"))):
        with open(os.path.join(ROOT, "paper_1805_09246_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


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


def cpu_baseline(stream, params, window, threshold, n_slices_sample=10, n_scans=10):
    """The oracle timed on the host on a bounded sample: ingest of the first slices, then a
    few scans; scaled to the whole job's packets/s."""
    import oracle
    threads = oracle.default_threads()
    o = oracle.OracleSketch(params)
    t0 = time.perf_counter()
    n_pk = 0
    for s in range(1, n_slices_sample + 1):
        p = stream.slice_pkts(s)
        o.ingest(p, s)
        n_pk += p.shape[0]
    t_ing = time.perf_counter() - t0
    t_scan = []
    for j in range(n_scans):
        s = n_slices_sample + j
        if j:
            p = stream.slice_pkts(s)
            t1 = time.perf_counter()
            o.ingest(p, s)
            t_ing += time.perf_counter() - t1
            n_pk += p.shape[0]
        t1 = time.perf_counter()
        o.scan(window, threshold, threads=threads)
        t_scan.append(time.perf_counter() - t1)
    per_pkt = t_ing / n_pk
    scan_s = sum(t_scan) / len(t_scan)
    rec = stream.recipe
    n_scans_job = rec.n_slices - window + 1
    job_s = per_pkt * rec.n_packets + scan_s * n_scans_job
    return {
        "value": rec.n_packets / job_s,
        "unit": "packets/s",
        "cores": threads,
        "kind": "oracle",
        "sample": (f"oracle ingest of slices 1..{n_slices_sample + n_scans - 1} "
                   f"({n_pk} packets, 1 thread, {t_ing:.2f} s) and {n_scans} scans "
                   f"(exhaustive candidate search on {threads} threads, "
                   f"{scan_s:.2f} s each), scaled to {rec.n_packets} packets and "
                   f"{n_scans_job} scans"),
        "ingest_pkts_per_s": 1.0 / per_pkt,
        "scan_ms_per_slice": scan_s * 1e3,
    }


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
        sps.sps_set_tuning(r.h, best["blocks_per_cu"], best["batch_tile"])
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


def serving_extra(pool, log_fn):
    """Config 4: the serving loop in real time; p50/p99 arrival-to-report latency."""
    import numpy as np
    from paper_1805_09246_amd.serve import Server, poisson_schedule, run_simulation
    from synth.configs import (C4_BUDGET, C4_PARAMS, C4_RATE, C4_ROUTERS, C4_SEED, C4_SLICE_S,
                               C4_SLICES, C4_THRESHOLD, C4_WINDOW)
    srv = Server(C4_PARAMS, C4_WINDOW, C4_THRESHOLD, C4_BUDGET)
    for r in range(C4_ROUTERS):
        srv.admit(r)
    sched = poisson_schedule(C4_SEED, C4_RATE, C4_SLICES * C4_SLICE_S, C4_ROUTERS)
    wall, n_pk = run_simulation(srv, pool, sched, C4_SLICE_S, C4_SLICES)
    lat = np.array([x for r in srv.reports for x in r.latencies])
    slices_done = max(r.slice for r in srv.reports)
    log_fn(f"serving: {len(lat)} batches, {n_pk} packets in {wall:.2f} s")
    out = {
        "workload": f"{C4_ROUTERS} routers, Poisson batches 4Ki-4Mi at {C4_RATE:.0e} pkt/s, "
                    f"{C4_SLICES} slices of {C4_SLICE_S * 1e3:.0f} ms, window {C4_WINDOW}",
        "packets_per_s": n_pk / wall,
        "offered_packets_per_s": C4_RATE,
        "batches": int(len(lat)),
        "p50_latency_ms": float(np.percentile(lat, 50) * 1e3),
        "p99_latency_ms": float(np.percentile(lat, 99) * 1e3),
        "max_latency_ms": float(lat.max() * 1e3),
        "slices": slices_done,
        "wall_s": wall,
        "resident_sketches": len(srv.slots),
        "resident_GiB": srv.used_bytes() / 2 ** 30,
    }
    for s in srv.slots:
        s.sketch.close()
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
    rec, params, K_WIN, THETA = C2_RECIPE, C2_PARAMS, C2_WINDOW, C2_THRESHOLD
    t0 = time.perf_counter()
    st = make_stream(rec)
    log(f"stream generated in {time.perf_counter() - t0:.1f} s")
    pkts = torch.from_numpy(st.pkts.view(np.int32)).cuda()
    offs = [int(v) for v in st.slice_off]
    slices = [pkts[offs[s - 1]:offs[s]] for s in range(1, rec.n_slices + 1)]
    sk = sps.Sketch(params)
    n_scans = rec.n_slices - K_WIN + 1
    cap = 8192
    res = torch.zeros((n_scans, cap * 24), dtype=torch.uint8, device="cuda")
    info = torch.zeros((n_scans, 8), dtype=torch.int32, device="cuda")

    def step():
        sk.reset()
        for s in range(1, rec.n_slices + 1):
            sps.sps_ingest(sk.h, slices[s - 1], s)
            if s >= K_WIN:
                j = s - K_WIN
                sps.sps_scan_async(sk.h, K_WIN, THETA, res[j], cap, info[j])

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    inf = info.cpu().numpy()
    if (inf[:, sps.INFO_FLAGS] != 0).any():
        raise RuntimeError("scan buffers overflowed")
    log(f"warm-up done; hosts reported per scan: {int(inf[:, 0].min())}..{int(inf[:, 0].max())}")
    # one profiled step with every kernel bracketed: the breakdown and the dominant kernel
    sps.sps_profile_enable(True)
    sps.sps_profile_read()
    step()
    prof_all = sps.sps_profile_read()
    kernel_stages = ("ingest", "scan_stats", "join", "estimate", "sort", "fill")
    dominant = max(kernel_stages, key=lambda k: prof_all[k][0])
    # timed region: events only around ingests, whole scans and the dominant kernel
    sps.sps_profile_enable(True, stages={"ingest", "scan", dominant})
    sps.sps_profile_read()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    prof = sps.sps_profile_read()
    sps.sps_profile_enable(False)
    log(f"timed {args.steps} steps in {elapsed:.3f} s; dominant kernel stage: {dominant}")

    total_pkts = args.steps * rec.n_packets
    value = total_pkts / elapsed
    tau, _, row_len = sk.derived()
    stores_per_pkt = params["rp"] + params["r"] * 2.0 ** -tau
    ingest_bytes_per_pkt = 8 + 2 * stores_per_pkt
    # a scan's first kernel streams the SLE array and the SRE array once
    stats_bytes = 2 * (params["rp"] * row_len + (params["r"] << params["q"]) * params["eta"]) \
        + (params["r"] << params["q"]) // 8
    # the candidate search: every expanded node tests its 2^delta extensions (Alg. 4-5), each
    # test a shift, xor, mask and bit test of 32-bit integers
    inf = info.cpu().numpy().astype(np.int64)
    nodes_per_scan = float(np.mean(inf[:, sps.INFO_NODES_LO] & 0xFFFFFFFF
                                   | (inf[:, sps.INFO_NODES_HI] << 32)))
    join_ops = nodes_per_scan * (1 << params["delta"]) * JOIN_OPS_PER_TEST
    stage_ms = {k: {"total_ms": round(v[0], 3), "launches": v[1],
                    "avg_us": round(1e3 * v[0] / v[1], 2) if v[1] else None}
                for k, v in prof_all.items() if v[1]}
    kernel_names = {"ingest": "k_ingest", "scan_stats": "k_scan_stats", "join": "k_join",
                    "estimate": "k_estimate", "sort": "k_rank_sort", "fill": "k_fill_zero"}

    def kernel_roofline(stage, avg_s):
        if stage in ("ingest", "scan_stats"):
            b = rec.n_packets / rec.n_slices * ingest_bytes_per_pkt if stage == "ingest" \
                else stats_bytes
            a = b / avg_s / 1e9
            return {"bound": "hbm", "achieved": round(a, 2), "peak": PEAK_HBM_GBS, "unit": "GB/s",
                    "frac": round(a / PEAK_HBM_GBS, 4), "alg_bytes_per_launch": int(b)}
        if stage == "join":
            a = join_ops / avg_s / 1e12
            return {"bound": "alu", "achieved": round(a, 4), "peak": PEAK_INT32_TOPS,
                    "unit": "Tops/s (int32 lane ops)", "frac": round(a / PEAK_INT32_TOPS, 4),
                    "nodes_per_launch": int(nodes_per_scan),
                    "alg_ops_per_launch": int(join_ops)}
        return None

    avg_s = prof[dominant][0] / prof[dominant][1] / 1e3
    roofline = kernel_roofline(dominant, avg_s) or {"bound": "alu", "achieved": None,
                                                     "peak": None, "unit": None, "frac": None}
    roofline.update({"traffic": stored_traffic(kernel_names[dominant]),
                     "kernel": kernel_names[dominant], "avg_launch_us": round(avg_s * 1e6, 2)})
    per_kernel = {}
    for k in ("ingest", "scan_stats", "join"):
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
        "ingest_pkts_per_s": total_pkts / (prof["ingest"][0] / 1e3),
        "scan_ms_per_slice": prof["scan"][0] / prof["scan"][1],
        "stage_ms_one_profiled_step": stage_ms,
        "per_kernel_roofline": per_kernel,
    }

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
        roof_pkts = 1.0 / (8.0 / BW_s + stores_per_pkt / R_s)
        ing = total_pkts / (prof["ingest"][0] / 1e3)
        out["roofline_measured"] = {
            "scatter_stores_per_s": R_s, "stream_GBps": BW_s / 1e9,
            "ingest_roofline_pkts_per_s": roof_pkts,
            "ingest_frac_of_measured": ing / roof_pkts,
            "scan_stats_frac_of_stream": (stats_bytes / (prof_all["scan_stats"][0] /
                                                         prof_all["scan_stats"][1] / 1e3)) / BW_s,
        }
        del probe

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
        out["cpu_baseline"] = cpu_baseline(st, params, K_WIN, THETA)
        log(f"cpu baseline in {time.perf_counter() - t0:.1f} s")

    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
