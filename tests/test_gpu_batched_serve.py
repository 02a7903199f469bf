"""Batched multi-router ingest, captured graphs, the autotuner, the distributed merge at the
multi-router workload's shapes, and the serving loop (GPU)."""
import numpy as np
import pytest
import torch

import oracle
from gpu_util import assert_results_equal, assert_scan_equal, assert_state_equal, dev_pkts
from paper_1805_09246_amd import sps
from paper_1805_09246_amd.serve import Server

pytestmark = pytest.mark.gpu

SMALL = dict(q=12, r=6, delta=5, eta=8, qp=8, rp=3, etap=64, deltap=16, theta=64, anet_side=0,
             seed=0xC0FFEE)


def _rand_pkts(rng, n, hosts=300):
    dst = (rng.zipf(1.3, n).astype(np.uint64) % hosts * 2654435761 + 12345).astype(np.uint32)
    src = rng.integers(0, 1 << 32, n, dtype=np.uint64).astype(np.uint32)
    return np.stack([src, dst], 1)


def test_graph_capture_replays_match_eager():
    rng = np.random.default_rng(1)
    eager, graphed = sps.Sketch(SMALL), sps.Sketch(SMALL)
    st = torch.cuda.Stream()
    out = torch.zeros(2048 * 24, dtype=torch.uint8, device="cuda")
    info = torch.zeros(8, dtype=torch.int32, device="cuda")
    for s in range(1, 6):
        p = dev_pkts(_rand_pkts(rng, 30000))
        eager.ingest(p, s)
        want = eager.scan(3, 20.0)
        with torch.cuda.stream(st):
            sps.sps_graph_begin(st)
            sps.sps_ingest(graphed.h, p, s, st)
            sps.sps_scan_async(graphed.h, 3, 20.0, out, 2048, info, st)
            g = sps.sps_graph_end(st)
            for rep in range(3):   # replays are idempotent; eager work in between
                sps.sps_graph_launch(g, st)
                st.synchronize()
                torch.zeros(1000, device="cuda").sum().item()
                n = int(info[sps.INFO_KEPT].item())
                got = out.cpu().numpy().view(sps.RESULT_DTYPE)[:n]
                assert np.array_equal(got, want), f"slice {s} replay {rep}"
            sps.sps_graph_destroy(g)
    assert np.array_equal(eager.export(), graphed.export())


@pytest.mark.parametrize("classes", [1, 2, 4, 8])
def test_ingest_host_classes_keep_state_exact(classes):
    """Every host-class partition of the ingest (and of the batched ingest) writes the same
    recorders: the state equals the oracle's."""
    rng = np.random.default_rng(20 + classes)
    a, b, c = sps.Sketch(SMALL), sps.Sketch(SMALL), sps.Sketch(SMALL)
    oa, ob, oc = (oracle.OracleSketch(SMALL) for _ in range(3))
    for g in (a, b, c):
        sps.sps_set_tuning(g.h, host_classes=classes)
    for s in (1, 2):
        pa, pb, pc = (_rand_pkts(rng, n) for n in (70000, 5000, 33000))
        a.ingest(dev_pkts(pa), s)
        sps.sps_ingest_batched([b.h, c.h], [dev_pkts(pb), dev_pkts(pc)], s)
        for o, p in ((oa, pa), (ob, pb), (oc, pc)):
            o.ingest(p, s)
    for g, o in ((a, oa), (b, ob), (c, oc)):
        assert_state_equal(g, o)


def test_autotune_keeps_state_exact():
    rng = np.random.default_rng(2)
    sizes = [100000, 3000, 0, 250000]
    gs = [sps.Sketch(SMALL) for _ in sizes]
    os_ = [oracle.OracleSketch(SMALL) for _ in sizes]
    for s in (1, 2):
        ps = [_rand_pkts(rng, n) for n in sizes]
        if s == 1:
            best, ms = sps.sps_autotune_ingest([g.h for g in gs], [dev_pkts(p) for p in ps], s)
            assert best["blocks_per_cu"] > 0 and min(ms) > 0
            assert len(ms) == sps.AUTOTUNE_CANDIDATES_BATCHED
            assert best["host_classes"] in (1, 8)
            assert sps.sps_get_tuning(gs[0].h) == best
            # the choice is in the tuning cache under this device's architecture
            assert sps.sps_tuning_lookup(SMALL, True) == best
        else:
            sps.sps_ingest_batched([g.h for g in gs], [dev_pkts(p) for p in ps], s)
        for o, p in zip(os_, ps):
            o.ingest(p, s)
    for g, o in zip(gs, os_):
        assert_state_equal(g, o)
    one = sps.Sketch(SMALL)
    p = _rand_pkts(rng, 50000)
    best, ms = sps.sps_autotune_ingest([one.h], [dev_pkts(p)], 3)
    assert len(ms) == sps.AUTOTUNE_CANDIDATES_SINGLE
    assert sps.sps_tuning_lookup(SMALL, False) == best
    o = oracle.OracleSketch(SMALL)
    o.ingest(p, 3)
    assert_state_equal(one, o)


def test_multi_router_merge_at_workload_shape():
    """16 routers with lognormal sizes ingested in one batched launch per slice, merged by
    max and scanned; equal to the oracle fed every router's packets (merge = union)."""
    from synth import make_multi_stream
    from synth.configs import C3_PARAMS, C3_SMALL_RECIPE
    rs = make_multi_stream(C3_SMALL_RECIPE)
    gs = [sps.Sketch(C3_PARAMS) for _ in rs]
    o = oracle.OracleSketch(C3_PARAMS)
    for s in range(1, C3_SMALL_RECIPE.n_slices + 1):
        ps = [r.slice_pkts(s) for r in rs]
        sps.sps_ingest_batched([g.h for g in gs], [dev_pkts(p) for p in ps], s)
        o.ingest(np.concatenate(ps), s)
    merged = sps.Sketch(C3_PARAMS)
    merged.merge(gs)
    assert_state_equal(merged, o, "merged")
    got = assert_scan_equal(merged, o, 10, 2048.0, "merged scan")
    assert set(rs[0].planted_hosts[1:].tolist()) <= set(got["host"].tolist())
    # a single router alone sees too few peers of the planted hosts
    alone = gs[0].scan(10, 2048.0)
    assert len(set(alone["host"]) & set(rs[0].planted_hosts.tolist())) < len(rs[0].planted_hosts)


def _serve(routers, schedule, n_slices, budget_sketches=8, use_graph=True):
    srv = Server(SMALL, window=3, threshold=20.0,
                 budget_bytes=budget_sketches * sps.sps_sketch_bytes(SMALL), use_graph=use_graph)
    for r in routers:
        srv.admit(r)
    for k in range(1, n_slices + 1):
        for (r, pk) in schedule.get(k, []):
            if r in routers:
                srv.submit(r, pk)
        srv.run_slice()
        srv.collect()
    srv.collect(block=True)
    return srv


def test_stream_host_time_marks_completion():
    """The stream's host notification fires after the work queued before it and stores a
    CLOCK_MONOTONIC time between the launch and the host's wait."""
    import time
    g = sps.Sketch(SMALL)
    rng = np.random.default_rng(9)
    st = torch.cuda.Stream()
    t = np.zeros(1, dtype=np.float64)
    t0 = time.clock_gettime(time.CLOCK_MONOTONIC)
    with torch.cuda.stream(st):
        g.ingest(dev_pkts(_rand_pkts(rng, 300000)), 1, st)
        sps.sps_stream_host_time(t, st)
    st.synchronize()
    t1 = time.clock_gettime(time.CLOCK_MONOTONIC)
    assert t0 <= t[0] <= t1


def test_serving_result_same_alone_and_in_mix():
    rng = np.random.default_rng(3)
    schedule = {}
    for k in range(1, 9):
        schedule[k] = [(r, dev_pkts(_rand_pkts(rng, int(rng.integers(100, 40000)))))
                       for r in range(6) for _ in range(int(rng.integers(0, 3)))]
    mix = _serve(list(range(6)), schedule, 8)
    for r in (0, 4):
        alone = _serve([r], schedule, 8, use_graph=(r == 0))
        a = [x for x in alone.reports if x.router == r]
        b = [x for x in mix.reports if x.router == r]
        assert len(a) == len(b) == 8
        for x, y in zip(a, b):
            assert x.slice == y.slice and x.batches == y.batches and x.packets == y.packets
            assert np.array_equal(x.results, y.results)
    # and every report equals the oracle fed that router's packets
    o = oracle.OracleSketch(SMALL)
    for k in range(1, 9):
        pk = [p.cpu().numpy().view(np.uint32) for (r, p) in schedule[k] if r == 4]
        if pk:
            o.ingest(np.concatenate(pk), k)
        else:
            o.set_slice(k)
        want, _ = o.scan(3, 20.0)
        got = [x for x in mix.reports if x.router == 4 and x.slice == k][0]
        assert got.complete
        assert_results_equal(got.results, want, f"served router 4, slice {k}")


def test_admission_by_budget_and_slot_reuse():
    rng = np.random.default_rng(4)
    srv = Server(SMALL, 3, 20.0, budget_bytes=2 * sps.sps_sketch_bytes(SMALL))
    assert srv.admit(10) and srv.admit(11)
    assert not srv.admit(12)                       # over budget: queued
    held = dev_pkts(_rand_pkts(rng, 5000))
    srv.submit(12, held)                           # held until admitted
    srv.run_slice()
    srv.collect(block=True)
    assert {r.router for r in srv.reports} == {10, 11}
    srv.release(10)                                # frees a slot; 12 takes it
    assert 12 in srv.by_router and len(srv.slots) == 2
    srv.run_slice()
    srv.collect(block=True)
    rep = [r for r in srv.reports if r.router == 12]
    assert len(rep) == 1 and rep[0].batches == 1 and rep[0].packets == 5000
    o = oracle.OracleSketch(SMALL)
    o.ingest(held.cpu().numpy().view(np.uint32), 2)
    want, _ = o.scan(3, 20.0)
    assert_results_equal(rep[0].results, want, "admitted router")


def test_serving_flags_truncated_reports():
    """A scan that keeps more hosts than the serving result buffer, or recovers more
    candidates than the sketch's candidate capacity, yields a report marked incomplete."""
    rng = np.random.default_rng(5)
    many = dev_pkts(_rand_pkts(rng, 200000, hosts=50))
    srv = Server(SMALL, 3, 1.0, budget_bytes=4 * sps.sps_sketch_bytes(SMALL), result_cap=2)
    srv.admit(1)
    srv.submit(1, many)
    srv.run_slice()
    srv.collect(block=True)
    rep = srv.reports[-1]
    assert rep.kept > 2 and len(rep.results) == 2 and not rep.complete
    assert rep.info_flags & 2 and srv.incomplete == 1
    tiny = dict(SMALL, cand_cap=4)
    srv2 = Server(tiny, 3, 1.0, budget_bytes=4 * sps.sps_sketch_bytes(tiny))
    srv2.admit(1)
    srv2.submit(1, many)
    srv2.run_slice()
    srv2.collect(block=True)
    assert srv2.reports[-1].info_flags & 1 and not srv2.reports[-1].complete


def test_serving_runs_past_slice_limit():
    """Serving started near the u16 limit rebases every resident sketch before slice 65535
    and goes on; every report equals the oracle fed that router's packets from slice 1."""
    rng = np.random.default_rng(6)
    routers = [0, 1, 2]
    srv = Server(SMALL, window=3, threshold=20.0,
                 budget_bytes=4 * sps.sps_sketch_bytes(SMALL), start_slice=65528)
    for r in routers:
        srv.admit(r)
    sent = {r: [] for r in routers}
    for k in range(1, 13):
        for r in routers:
            p = _rand_pkts(rng, int(rng.integers(500, 20000)))
            sent[r].append(p)
            srv.submit(r, dev_pkts(p))
        srv.run_slice()
        srv.collect()
    srv.collect(block=True)
    assert srv.rebases == 1 and srv.slice_no < 65534
    for r in routers:
        o = oracle.OracleSketch(SMALL)
        reps = sorted((x for x in srv.reports if x.router == r), key=lambda x: x.slice)
        assert [x.slice for x in reps] == list(range(65529, 65541))
        for k, (p, rep) in enumerate(zip(sent[r], reps), 1):
            o.ingest(p, k)
            want, _ = o.scan(3, 20.0)
            assert rep.complete
            assert_results_equal(rep.results, want, f"router {r}, slice {rep.slice}")
