"""GPU parity on the paths the workload streams rarely reach: every ordering path of the
final report (Sec. 4 end: the kept hosts ascending), the join's per-block candidate buffer
overflowing into the global list, and the join's 64-bit pair arithmetic when rows 0 and 1
have more than 2^32 pairs (Alg. 4-5).  Compared with the oracle element by element."""
import numpy as np
import pytest
import torch

import oracle
from gpu_util import (assert_results_equal, assert_scan_equal, assert_state_equal, dev_pkts,
                      gpu_candidates, gpu_hot, gpu_row_live, import_state)
from paper_1805_09246_amd import sps

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _device():
    torch.cuda.set_device(0)
    yield
    torch.cuda.synchronize()


def _hosts_with_peers(n_hosts, peers, seed):
    rng = np.random.default_rng(seed)
    hosts = rng.choice(1 << 32, n_hosts, replace=False).astype(np.uint32)
    dst = np.repeat(hosts, peers)
    src = rng.integers(0, 1 << 32, dst.size, dtype=np.uint64).astype(np.uint32)
    return np.stack([src, dst], 1)


ORDER = dict(q=17, r=10, delta=2, eta=8, qp=12, rp=3, etap=64, deltap=64, theta=8,
             anet_side=0, seed=41)


@pytest.mark.parametrize("n_hosts", [1100, 3000, 4096, 4097, 10000])
def test_report_order_paths(n_hosts):
    """1100, 3000 and 4096 kept hosts: one block sorts them with two (1100) or four keys per
    thread, padded above the hosts (3000); 4097 and 10000: 4096-key tiles sorted by every
    block, then placed by rank.  Every host has 12 peers (tau = 0, so all are
    sampled) and is reported; the whole report equals the oracle's."""
    p = _hosts_with_peers(n_hosts, 12, n_hosts)
    g, o = sps.Sketch(ORDER), oracle.OracleSketch(ORDER)
    g.ingest(dev_pkts(p), 1)
    o.ingest(p, 1)
    print(f"[order] {n_hosts} hosts ingested", flush=True)
    got = assert_scan_equal(g, o, 1, 4.0, f"{n_hosts} hosts")
    assert len(got) == n_hosts
    g.close()


@pytest.mark.parametrize("cand_cap", [1100, 1107])
def test_report_at_candidate_capacity(cand_cap):
    """1100 candidates, all kept: a candidate list and kept list exactly as long as the
    capacity (and one 7 entries longer) give the oracle's full report without overflow."""
    p = _hosts_with_peers(1100, 12, 1100)
    params = dict(ORDER, cand_cap=cand_cap)
    g, o = sps.Sketch(params), oracle.OracleSketch(params)
    g.ingest(dev_pkts(p), 1)
    o.ingest(p, 1)
    got = assert_scan_equal(g, o, 1, 4.0, f"cand_cap {cand_cap}")
    assert len(got) == 1100
    g.close()


@pytest.mark.parametrize("n_kept,n_dropped,cand_cap", [(2000, 1000, 3100), (4500, 1500, 6200)])
def test_report_from_multi_entry_kept_regions(n_kept, n_dropped, cand_cap):
    """More candidates than the estimate's 2048 waves, at capacities that give every wave a
    kept-list region of 2 (4) entries, with candidates the filter drops mixed in (hosts with
    4 peers are hot enough to be recovered but estimate below 8): the report, ordered in LDS
    (2000 kept) or by tiles and ranks (4500 kept), equals the oracle's."""
    rng = np.random.default_rng(n_kept)
    hosts = rng.choice(1 << 32, n_kept + n_dropped, replace=False).astype(np.uint32)
    dst = np.concatenate([np.repeat(hosts[:n_kept], 12), np.repeat(hosts[n_kept:], 4)])
    src = rng.integers(0, 1 << 32, dst.size, dtype=np.uint64).astype(np.uint32)
    p = np.stack([src, dst], 1)[rng.permutation(dst.size)]
    params = dict(ORDER, cand_cap=cand_cap)
    g, o = sps.Sketch(params), oracle.OracleSketch(params)
    g.ingest(dev_pkts(p), 1)
    o.ingest(p, 1)
    print(f"[kept regions] {n_kept} + {n_dropped} hosts ingested, cand_cap {cand_cap}", flush=True)
    got = assert_scan_equal(g, o, 1, 8.0, f"{n_kept} kept of {n_kept + n_dropped}")
    assert len(got) > (4096 if n_kept > 4096 else 1024)  # the ordering path named above
    g.close()


def _crafted(params, hot_cols, cur=3, seed=0):
    """SRE state whose hot SREs are exactly hot_cols[i] in row i (three cells stamped `cur`,
    the hot cut for eta = 8), SLE array empty; the same state in a GPU and an oracle sketch."""
    p = params
    sre = np.zeros((p["r"], 1 << p["q"], p["eta"]), np.uint16)
    for i, cols in enumerate(hot_cols):
        sre[i, np.asarray(cols, np.int64), :3] = cur
    g, o = sps.Sketch(params), oracle.OracleSketch(params)
    row_len = (1 << p["qp"]) * p["deltap"] + p["etap"] - p["deltap"]
    import_state(g, sre, np.zeros((p["rp"], row_len), np.uint16), cur)
    o.sre()[...] = sre
    assert o.set_slice(cur) == 0
    return g, o


def test_join_block_candidate_buffer_overflows():
    """One hot SRE in rows 0 and 1 and half of rows 2-7 hot at q = 6, delta = 5: every
    candidate comes from the single pair (he0, he1), so one block finds thousands of them and
    its LDS buffer (1024 entries) spills into the global list.  The pair's subtree also
    outgrows the wave's stack (per-lane depth-first search)."""
    params = dict(q=6, r=8, delta=5, eta=8, qp=4, rp=2, etap=16, deltap=16, theta=8,
                  anet_side=0, seed=44, cand_cap=1 << 16)
    rng = np.random.default_rng(2)
    hot = [[17], [40]] + [np.flatnonzero(rng.random(64) < 0.5) for _ in range(6)]
    g, o = _crafted(params, hot)
    assert_scan_equal(g, o, 1, 1e9, "single-pair candidates")
    n = len(gpu_candidates(g))
    print(f"[overflow] {n} candidates from one pair", flush=True)
    assert n > 4 * 1024
    g.close()


def _wide_rows(rng, params, n_hot):
    return [rng.choice(1 << params["q"], n_hot, replace=False) for _ in range(2)]


WIDE = dict(q=17, r=10, delta=2, eta=8, qp=4, rp=2, etap=16, deltap=16, theta=8, anet_side=0,
            seed=45)


def test_join_pairs_beyond_32_bits_all_visited():
    """70000 hot SREs in rows 0 and 1 (4.9e9 pairs, more than 2^32) and an empty row 2: no
    pair extends, so the search expands exactly one node per pair.  The node count must be
    n0 * n1: every pair number past 2^32 is turned into (a, b) exactly once."""
    rng = np.random.default_rng(3)
    rows01 = _wide_rows(rng, WIDE, 70000)
    g, o = _crafted(WIDE, rows01 + [[] for _ in range(8)])
    d_out = torch.empty(1024 * 24, dtype=torch.uint8, device="cuda")
    d_info = torch.zeros(sps.INFO_WORDS, dtype=torch.int32, device="cuda")
    sps.sps_scan_async(g.h, 1, 1e9, d_out, 1024, d_info)
    torch.cuda.synchronize()
    inf = d_info.cpu().numpy().view(np.uint32)
    nodes = int(inf[sps.INFO_NODES_LO]) | (int(inf[sps.INFO_NODES_HI]) << 32)
    assert int(inf[sps.INFO_HSE0]) == 70000 and int(inf[sps.INFO_HSE1]) == 70000
    assert nodes == 70000 * 70000 > (1 << 32)
    assert int(inf[sps.INFO_CAND]) == 0
    g.close()


def test_join_pairs_beyond_32_bits_find_planted():
    """The same wide rows 0 and 1, and rows 2-9 hot only where 40 chosen addresses land:
    the candidates (found through 64-bit pair numbers) equal the oracle's exhaustive search
    and include the chosen addresses."""
    rng = np.random.default_rng(4)
    rows01 = _wide_rows(rng, WIDE, 70000)
    probe = oracle.OracleSketch(WIDE)
    xs = rng.integers(0, 1 << 32, 40, dtype=np.uint64).astype(np.uint32)
    hot = [list(r) for r in rows01] + [[] for _ in range(8)]
    for x in xs.tolist():
        for i in range(WIDE["r"]):
            hot[i].append(probe.hash(probe.RHFG, i, x))
    hot = [np.unique(np.asarray(h, np.int64)) for h in hot]
    g, o = _crafted(WIDE, hot)
    got = assert_scan_equal(g, o, 1, -1.0, "wide rows, planted addresses")
    assert set(xs.tolist()) <= set(gpu_candidates(g).tolist())
    assert len(got) == len(gpu_candidates(g))  # a negative threshold keeps every candidate
    g.close()


def test_c4_sketch_shape_parity():
    """The serving workload's sketch shape (SLE array 5 x 16384 x 1024) on the small stream of
    the scale workload, fed through the batched ingest as four routers: each router's state,
    the merged state and the merged scans equal the oracle's."""
    from synth import make_stream
    from synth.configs import C2_SMALL_RECIPE, C4_PARAMS, C4_THRESHOLD, C4_WINDOW
    st = make_stream(C2_SMALL_RECIPE)
    rng = np.random.default_rng(6)
    gs = [sps.Sketch(C4_PARAMS) for _ in range(4)]
    os_ = [oracle.OracleSketch(C4_PARAMS) for _ in range(4)]
    whole = oracle.OracleSketch(C4_PARAMS)
    merged = sps.Sketch(C4_PARAMS)
    for s in range(1, st.recipe.n_slices + 1):
        p = st.slice_pkts(s)
        who = rng.integers(0, 4, len(p))
        parts = [p[who == j] for j in range(4)]
        sps.sps_ingest_batched([g.h for g in gs], [dev_pkts(x) for x in parts], s)
        for o, x in zip(os_, parts):
            o.ingest(x, s)
        whole.ingest(p, s)
        if s >= C4_WINDOW:
            merged.merge(gs)
            assert_state_equal(merged, whole, f"merged at slice {s}")
            got = assert_scan_equal(merged, whole, C4_WINDOW, C4_THRESHOLD, f"slice {s}")
            print(f"[c4 shape] slice {s}: {len(got)} hosts", flush=True)
    for j, (g, o) in enumerate(zip(gs, os_)):
        assert_state_equal(g, o, f"router {j}")
        assert_scan_equal(g, o, C4_WINDOW, C4_THRESHOLD, f"router {j}")


@pytest.mark.slow
def test_c3_full_size_merged_scans():
    """The distributed-merge workload at full size (16 routers, lognormal sizes around 2^22
    packets, 30 slices): routers fed by the batched ingest, merged by max after slices 20 and
    30; the merged state and its scan (window 10, threshold 2048) equal an oracle sketch fed
    every router's packets (the merge is the union, Alg. 2 / Alg. 7)."""
    from synth import make_multi_stream
    from synth.configs import C3_PARAMS, C3_RECIPE, C3_THRESHOLD, C3_WINDOW
    rs = make_multi_stream(C3_RECIPE)
    print(f"[c3] {sum(r.pkts.shape[0] for r in rs)} packets generated", flush=True)
    gs = [sps.Sketch(C3_PARAMS) for _ in rs]
    o = oracle.OracleSketch(C3_PARAMS)
    merged = sps.Sketch(C3_PARAMS)
    for s in range(1, C3_RECIPE.n_slices + 1):
        ps = [r.slice_pkts(s) for r in rs]
        sps.sps_ingest_batched([g.h for g in gs], [dev_pkts(p) for p in ps], s)
        o.ingest(np.concatenate(ps), s)
        if s in (20, 30):
            merged.merge(gs)
            assert_state_equal(merged, o, f"merged at slice {s}")
            got = assert_scan_equal(merged, o, C3_WINDOW, C3_THRESHOLD, f"c3 scan at {s}")
            print(f"[c3] slice {s}: state equal, {len(got)} hosts reported", flush=True)
            assert len(got) > 1024  # the ordering takes its LDS path at this size
    for g in gs:
        g.close()
    merged.close()


def test_saturated_sre_array_skips_the_search():
    """Every SRE hot in every row (all pairs sampled, hundreds per SRE): the expected search
    passes 2^36 nodes, so the search is not run and the scan reports a candidate overflow at
    once (flags bits 0 and 2) instead of running for seconds; a row-count scan of the same
    sketch with a short window that leaves it unsaturated still matches the oracle."""
    import time
    params = dict(q=12, r=6, delta=5, eta=8, qp=10, rp=2, etap=64, deltap=64, theta=8,
                  anet_side=0, seed=43)
    rng = np.random.default_rng(43)
    g = sps.Sketch(params)
    o = oracle.OracleSketch(params)
    p = rng.integers(0, 1 << 32, size=(2_000_000, 2), dtype=np.uint64).astype(np.uint32)
    g.ingest(dev_pkts(p), 1)
    o.ingest(p, 1)
    hot = o.hot(1)
    assert hot.mean() > 0.99  # the oracle agrees the array is saturated
    out = torch.zeros(4096 * 24, dtype=torch.uint8, device="cuda")
    info = torch.zeros(8, dtype=torch.int32, device="cuda")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sps.sps_scan_async(g.h, 1, 8.0, out, 4096, info)
    torch.cuda.synchronize()
    assert time.perf_counter() - t0 < 2.0
    f = int(info[sps.INFO_FLAGS].item())
    assert f & 1 and f & 4 and int(info[sps.INFO_KEPT].item()) == 0
    with pytest.raises(sps.SpsError) as e:
        g.scan(1, 8.0)
    assert e.value.code == sps.SPS_ECAPACITY
    # the row-count sweep still ran in the skipped search's launch
    assert np.array_equal(gpu_row_live(g), o.row_live(1)), "row live counts of the skipped scan"
    # a later, unsaturated window of the same sketch is searched as usual
    q = rng.integers(0, 1 << 32, size=(3000, 2), dtype=np.uint64).astype(np.uint32)
    g.ingest(dev_pkts(q), 2)
    o.ingest(q, 2)
    assert_scan_equal(g, o, 1, 8.0, "after saturation")
    g.close()


# (q, r, delta): the hot-SRE pass by tiles of 2^(delta+6) SREs (q - delta >= 6; delta 1 leaves
# waves of the block idle, delta 5 gives each wave 8 groups, q - delta = 6 one tile per row),
# else one SRE per lane with atomic table bits (q - delta < 6)
SRE_SHAPES = [(7, 27, 1), (8, 26, 1), (9, 10, 3), (10, 8, 4), (11, 7, 5), (14, 11, 2),
              (8, 10, 3)]


@pytest.mark.parametrize("shape", SRE_SHAPES, ids=lambda s: f"q{s[0]}r{s[1]}d{s[2]}")
def test_sre_pass_shapes_and_sweep_modes(shape):
    """Hot bitmap, row live counts, candidates and reports equal the oracle's across the tile
    shapes of the hot-SRE pass and its one-SRE-per-lane fallback, with the row-count sweep in
    the search's launch (scan_overlap 1) and after it (2)."""
    q, r, delta = shape
    params = dict(q=q, r=r, delta=delta, eta=8, qp=10, rp=3, etap=64, deltap=64, theta=64,
                  anet_side=0, seed=1000 * q + delta)
    rng = np.random.default_rng(17 * q + delta)
    gs = [sps.Sketch(params), sps.Sketch(params)]
    sps.sps_set_tuning(gs[0].h, scan_overlap=1)
    sps.sps_set_tuning(gs[1].h, scan_overlap=2)
    o = oracle.OracleSketch(params)
    hosts = rng.integers(0, 1 << 32, size=6, dtype=np.uint64).astype(np.uint32)
    for s in (1, 2):
        src = rng.integers(0, 1 << 32, size=6 * 150, dtype=np.uint64).astype(np.uint32)
        planted = np.stack([src, np.repeat(hosts, 150)], 1)
        noise = rng.integers(0, 1 << 32, size=(1500, 2), dtype=np.uint64).astype(np.uint32)
        p = np.concatenate([planted, noise])
        print(f"sre pass q={q} r={r} delta={delta} slice {s}", flush=True)
        for g in gs:
            g.ingest(dev_pkts(p), s)
        o.ingest(p, s)
        want, ocand = o.scan(2, 64.0)
        assert np.isin(hosts, want["host"]).all()  # the planted hosts are found
        for mode, g in zip((1, 2), gs):
            where = f"q{q} r{r} delta{delta} mode {mode} slice {s}"
            got = g.scan(2, 64.0, cap=1 << 18)
            assert np.array_equal(gpu_row_live(g), o.row_live(2)), f"{where}: row live counts"
            assert np.array_equal(gpu_hot(g), o.hot(2)), f"{where}: hot SREs"
            assert np.array_equal(gpu_candidates(g), ocand), f"{where}: candidates"
            assert_results_equal(got, want, where)
    for g in gs:
        g.close()
