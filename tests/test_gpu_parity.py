"""GPU parity: the HIP path, called through the C ABI, against the CPU oracle.

Sketch state, hot SREs, row live counts and candidate lists must be bit-exact; estimates
within 4 ulp (fp64, device log1p vs glibc); reported hosts, |USLE|^k and flags exact.
"""
import dataclasses

import numpy as np
import pytest
import torch

import oracle
from gpu_util import (assert_estimates_close, assert_scan_equal, assert_state_equal,
                      dev_pkts, gpu_candidates, gpu_hot)
from paper_1805_09246_amd import sps

pytestmark = pytest.mark.gpu

SMALL = dict(q=12, r=6, delta=5, eta=8, qp=8, rp=3, etap=64, deltap=16, theta=64, anet_side=0,
             seed=0xC0FFEE)


def _rand_pkts(rng, n, hosts=300, zipf=1.3):
    dst = (rng.zipf(zipf, n).astype(np.uint64) % hosts * 2654435761 + 12345).astype(np.uint32)
    src = rng.integers(0, 1 << 32, n, dtype=np.uint64).astype(np.uint32)
    return np.stack([src, dst], 1)


@pytest.fixture(scope="module", autouse=True)
def _device():
    torch.cuda.set_device(0)
    print(f"[gpu] {torch.cuda.get_device_name(0)}", flush=True)
    yield
    torch.cuda.synchronize()


def test_c1_full_stream(c1_stream):
    """Config 1 (2^20 packets, 10 slices, window 5, threshold 1024): state after every slice
    and the scan after every full window."""
    from synth.configs import C1_PARAMS, C1_THRESHOLD, C1_WINDOW
    g = sps.Sketch(C1_PARAMS)
    o = oracle.OracleSketch(C1_PARAMS)
    assert g.derived() == (o.tau, o.hot_cut, o.row_len)
    for s in range(1, 11):
        p = c1_stream.slice_pkts(s)
        g.ingest(dev_pkts(p), s)
        assert o.ingest(p, s) == 0
        assert_state_equal(g, o, f"slice {s}")
        if s >= C1_WINDOW:
            got = assert_scan_equal(g, o, C1_WINDOW, C1_THRESHOLD, f"scan at slice {s}")
            print(f"[c1] slice {s}: {len(got)} hosts reported", flush=True)
    g.close()


def test_scan_sweep_inside_and_after_the_search(c1_stream):
    """The row-count sweep inside the candidate search's launch (the default) and as a kernel
    of its own after the search give the oracle's scans."""
    from synth.configs import C1_PARAMS, C1_THRESHOLD, C1_WINDOW
    g, h = sps.Sketch(C1_PARAMS), sps.Sketch(C1_PARAMS)
    assert sps.sps_get_scan_overlap(g.h)
    sps.sps_set_tuning(h.h, scan_overlap=2)
    assert not sps.sps_get_scan_overlap(h.h)
    o = oracle.OracleSketch(C1_PARAMS)
    for s in range(1, 8):
        p = c1_stream.slice_pkts(s)
        g.ingest(dev_pkts(p), s)
        h.ingest(dev_pkts(p), s)
        o.ingest(p, s)
        if s >= C1_WINDOW:
            assert_scan_equal(g, o, C1_WINDOW, C1_THRESHOLD, f"sweep in the search, slice {s}")
            assert_scan_equal(h, o, C1_WINDOW, C1_THRESHOLD, f"sweep after the search, slice {s}")
    g.close()
    h.close()


@pytest.mark.parametrize("n", [0, 1, 63, 64, 65, 257, 4097, 100003])
def test_ragged_batch_sizes(n):
    rng = np.random.default_rng(n + 1)
    g, o = sps.Sketch(SMALL), oracle.OracleSketch(SMALL)
    for s in (1, 2):
        p = _rand_pkts(rng, n)
        g.ingest(dev_pkts(p), s)
        o.ingest(p, s)
    assert_state_equal(g, o, f"n={n}")
    assert_scan_equal(g, o, 2, 40.0, f"n={n}")


SHAPES = [
    dict(SMALL),                                           # shared SLE cells (delta' < eta')
    dict(SMALL, deltap=64),                                # no sharing
    dict(SMALL, anet_side=1),                              # aip = src
    dict(SMALL, eta=16, theta=128),                        # 16-cell SREs, hot cut 5
    dict(SMALL, rp=1, deltap=1),                           # one SLE row, densest sharing
    dict(SMALL, q=10, r=7, delta=5),                       # 35-bit coverage
    dict(SMALL, q=14, r=11, delta=2, qp=10, rp=8),         # config-2 SRE shape, 8 SLE rows
    dict(SMALL, etap=2048, deltap=2048, qp=6, theta=16),   # eta' > 1024, tau = 1
]


@pytest.mark.parametrize("params", SHAPES, ids=lambda p: f"q{p['q']}r{p['r']}e{p['eta']}"
                         f"rp{p['rp']}ep{p['etap']}dp{p['deltap']}s{p['anet_side']}")
def test_shapes(params):
    rng = np.random.default_rng(params["q"] * 7 + params["rp"])
    g, o = sps.Sketch(params), oracle.OracleSketch(params)
    for s in (1, 2, 3, 5, 6):
        p = _rand_pkts(rng, 20000, hosts=200, zipf=1.2)
        g.ingest(dev_pkts(p), s)
        o.ingest(p, s)
    assert_state_equal(g, o)
    for k in (1, 3, 6, 100):
        assert_scan_equal(g, o, k, 30.0, f"k={k}")


def test_merge_parity_and_union():
    rng = np.random.default_rng(3)
    n_r = 4
    gs = [sps.Sketch(SMALL) for _ in range(n_r)]
    os_ = [oracle.OracleSketch(SMALL) for _ in range(n_r)]
    whole = sps.Sketch(SMALL)
    for s in (1, 2, 4):
        p = _rand_pkts(rng, 30000)
        who = rng.integers(0, n_r, len(p))
        whole.ingest(dev_pkts(p), s)
        for j in range(n_r):
            gs[j].ingest(dev_pkts(p[who == j]), s)
            os_[j].ingest(p[who == j], s)
    gm, om = sps.Sketch(SMALL), oracle.OracleSketch(SMALL)
    gm.merge(gs)
    om.merge(os_)
    assert_state_equal(gm, om, "merged")
    # union: merging the routers equals one sketch fed everything
    ws, wl = whole.state()
    ms, ml = gm.state()
    assert np.array_equal(ws, ms) and np.array_equal(wl, ml)
    assert_scan_equal(gm, om, 3, 40.0, "merged scan")
    # accumulate into a router that is also a source
    gs[0].merge(gs[1:] + [gs[0]])
    s0, l0 = gs[0].state()
    assert np.array_equal(s0, ms) and np.array_equal(l0, ml)


def test_batched_ingest_parity():
    rng = np.random.default_rng(5)
    sizes = [0, 1, 5000, 70001, 300, 4096, 4097]
    gs = [sps.Sketch(SMALL) for _ in sizes]
    os_ = [oracle.OracleSketch(SMALL) for _ in sizes]
    for s in (1, 2, 3):
        ps = [_rand_pkts(rng, n) for n in sizes]
        sps.sps_ingest_batched([g.h for g in gs], [dev_pkts(p) for p in ps], s)
        for o, p in zip(os_, ps):
            o.ingest(p, s)
    for j, (g, o) in enumerate(zip(gs, os_)):
        assert_state_equal(g, o, f"router {j}")


def test_export_import_reset_resume():
    rng = np.random.default_rng(7)
    a, o = sps.Sketch(SMALL), oracle.OracleSketch(SMALL)
    pk = [_rand_pkts(rng, 8000) for _ in range(4)]
    for s in (1, 2):
        a.ingest(dev_pkts(pk[s - 1]), s)
        o.ingest(pk[s - 1], s)
    dump = a.export()
    b = sps.Sketch(SMALL)
    b.import_(dump)
    assert b.cur == 2
    for s in (3, 4):   # resume both
        a.ingest(dev_pkts(pk[s - 1]), s)
        b.ingest(dev_pkts(pk[s - 1]), s)
        o.ingest(pk[s - 1], s)
    assert_state_equal(b, o, "resumed")
    assert np.array_equal(a.export(), b.export())
    a.reset()
    sre, slea = a.state()
    assert a.cur == 0 and not sre.any() and not slea.any()
    other = sps.Sketch(dict(SMALL, seed=1))
    with pytest.raises(sps.SpsError) as e:
        other.import_(dump)
    assert e.value.code == sps.SPS_EMISMATCH


def test_features_parity(c1_stream):
    from synth.configs import C1_PARAMS
    g, o = sps.Sketch(C1_PARAMS), oracle.OracleSketch(C1_PARAMS)
    for s in range(1, 8):
        p = c1_stream.slice_pkts(s)
        g.ingest(dev_pkts(p), s)
        o.ingest(p, s)
    rng = np.random.default_rng(0)
    hosts = np.concatenate([c1_stream.planted_hosts,
                            rng.integers(0, 1 << 32, 500, dtype=np.uint64).astype(np.uint32),
                            c1_stream.pkts[:300, 1]])
    hd = torch.from_numpy(hosts.view(np.int32)).cuda()
    for k in (1, 5, 10, 32):
        x = g.features(hd, k).cpu().numpy().view(np.uint32)
        assert np.array_equal(x, o.features(k, hosts)), f"k={k}"
    with pytest.raises(sps.SpsError):
        g.features(hd, 33)


def test_error_paths():
    rng = np.random.default_rng(9)
    g = sps.Sketch(SMALL)
    p = dev_pkts(_rand_pkts(rng, 100))
    for bad in (0, 65535):
        with pytest.raises(sps.SpsError) as e:
            g.ingest(p, bad)
        assert e.value.code == sps.SPS_ESLICE
    g.ingest(p, 5)
    with pytest.raises(sps.SpsError) as e:
        g.ingest(p, 4)
    assert e.value.code == sps.SPS_ESLICE
    with pytest.raises(sps.SpsError) as e:
        g.merge([sps.Sketch(dict(SMALL, seed=2))])
    assert e.value.code == sps.SPS_EMISMATCH
    with pytest.raises(sps.SpsError) as e:
        sps.sps_ingest_batched([g.h, sps.Sketch(dict(SMALL, seed=2)).h], [p, p], 6)
    assert e.value.code == sps.SPS_EMISMATCH
    with pytest.raises(sps.SpsError) as e:
        g.scan(0, 10.0)
    assert e.value.code == sps.SPS_EINVAL
    g.advance(7)
    assert g.cur == 7
    # result capacity: required count reported, retry gives the same list
    many = dev_pkts(_rand_pkts(rng, 200000, hosts=50, zipf=1.01))
    g.ingest(many, 8)
    full = g.scan(2, 1.0)
    assert len(full) > 2
    with pytest.raises(sps.SpsError) as e:
        g.scan(2, 1.0, cap=2)
    assert e.value.code == sps.SPS_ECAPACITY and f"required {len(full)}" in str(e.value)
    again = g.scan(2, 1.0)
    assert np.array_equal(again, full)


def test_candidate_overflow():
    rng = np.random.default_rng(10)
    g = sps.Sketch(dict(SMALL, cand_cap=4))
    g.ingest(dev_pkts(_rand_pkts(rng, 200000, hosts=50, zipf=1.01)), 1)
    with pytest.raises(sps.SpsError) as e:
        g.scan(1, 1.0)
    assert e.value.code == sps.SPS_ECAPACITY


def test_scan_async_matches_sync(c1_stream):
    from synth.configs import C1_PARAMS
    g = sps.Sketch(C1_PARAMS)
    for s in range(1, 6):
        g.ingest(dev_pkts(c1_stream.slice_pkts(s)), s)
    sync = g.scan(5, 1024.0)
    out = torch.zeros(4096 * 24, dtype=torch.uint8, device="cuda")
    info = torch.zeros(8, dtype=torch.int32, device="cuda")
    sps.sps_scan_async(g.h, 5, 1024.0, out, 4096, info)
    torch.cuda.synchronize()
    inf = info.cpu().numpy()
    res = out.cpu().numpy().view(sps.RESULT_DTYPE)[: inf[sps.INFO_KEPT]]
    assert np.array_equal(res, sync)
    assert inf[sps.INFO_CAND] >= inf[sps.INFO_KEPT] and inf[sps.INFO_FLAGS] == 0


def test_launch_geometry_invariance():
    """Different packet splits and orders give identical state (Sec. 3.3: no sync needed)."""
    rng = np.random.default_rng(11)
    p = _rand_pkts(rng, 50000)
    a, b = sps.Sketch(SMALL), sps.Sketch(SMALL)
    a.ingest(dev_pkts(p), 1)
    q = p[rng.permutation(len(p))]
    for part in np.array_split(q, 7):
        b.ingest(dev_pkts(part), 1)
    assert np.array_equal(a.export(), b.export())


@pytest.mark.slow
def test_c2_full_size():
    """Config 2 at full size (2^26 packets, 60 slices, window 10): whole state after slices
    10, 35 and 60 and the full scan there."""
    from synth import make_stream
    from synth.configs import C2_PARAMS, C2_RECIPE, C2_THRESHOLD, C2_WINDOW
    st = make_stream(C2_RECIPE)
    print("[c2] stream generated", flush=True)
    g, o = sps.Sketch(C2_PARAMS), oracle.OracleSketch(C2_PARAMS)
    for s in range(1, 61):
        p = st.slice_pkts(s)
        g.ingest(dev_pkts(p), s)
        o.ingest(p, s)
        if s in (10, 35, 60):
            assert_state_equal(g, o, f"slice {s}")
            got = assert_scan_equal(g, o, C2_WINDOW, C2_THRESHOLD, f"c2 scan at {s}")
            print(f"[c2] slice {s}: state equal, {len(got)} hosts", flush=True)
    g.close()


def test_join_dense_rows_stack_fallback():
    """Rows about a quarter hot at q = 6, delta = 5 (32 extensions per node): the candidate
    search outgrows a wave's LDS stack, so batches fall back to per-lane depth-first search;
    candidates and results still match the oracle's exhaustive search."""
    params = dict(q=6, r=8, delta=5, eta=8, qp=8, rp=2, etap=64, deltap=64, theta=64,
                  anet_side=0, seed=77)
    rng = np.random.default_rng(5)
    n = 2 * 64 * 8
    hosts = rng.integers(0, 1 << 32, 40, dtype=np.uint64).astype(np.uint32)
    p = rng.integers(0, 1 << 32, size=(n, 2), dtype=np.uint64).astype(np.uint32)
    p[: n // 2, 1] = hosts[rng.integers(0, 40, n // 2)]
    g, o = sps.Sketch(params), oracle.OracleSketch(params)
    g.ingest(dev_pkts(p), 1)
    o.ingest(p, 1)
    assert_scan_equal(g, o, 1, 64.0, "dense rows")
    assert len(gpu_candidates(g)) > 10000


def _dense_sketch(params, n_pkts, n_hosts, seed):
    """Random peers towards few hosts: about a quarter to a half of every SRE row hot."""
    rng = np.random.default_rng(seed)
    hosts = rng.integers(0, 1 << 32, n_hosts, dtype=np.uint64).astype(np.uint32)
    p = rng.integers(0, 1 << 32, size=(n_pkts, 2), dtype=np.uint64).astype(np.uint32)
    p[:, 1] = hosts[rng.integers(0, n_hosts, n_pkts)]
    g, o = sps.Sketch(params), oracle.OracleSketch(params)
    g.ingest(dev_pkts(p), 1)
    o.ingest(p, 1)
    return g, o


def _join_nodes(g, k, threshold, cap=1 << 18):
    d_out = torch.empty(cap * 24, dtype=torch.uint8, device="cuda")
    d_info = torch.zeros(sps.INFO_WORDS, dtype=torch.int32, device="cuda")
    sps.sps_scan_async(g.h, k, threshold, d_out, cap, d_info)
    torch.cuda.synchronize()
    inf = d_info.cpu().numpy().view(np.uint32)
    return int(inf[sps.INFO_NODES_LO]) | (int(inf[sps.INFO_NODES_HI]) << 32)


DENSE_D2 = [  # delta = 2, rows dense enough that rows 1-3 are searched in bulk
    (dict(q=10, r=13), 15000, 1000),  # a quarter hot, coverage exactly 32 bits
    (dict(q=10, r=14), 10000, 1000),  # 34 bits: the top row's extensions must stay below 2^32
    (dict(q=12, r=12), 40000, 4000),  # 15 % hot
    (dict(q=10, r=13), 20000, 1000),  # a third hot: batches outgrow the stack, per-lane search
    (dict(q=8, r=14), 4000, 300),     # q < 10: the ordinary search on the same kind of rows
]


@pytest.mark.parametrize("shape,n_pkts,n_hosts", DENSE_D2,
                         ids=[f"q{s['q']}r{s['r']}n{n}" for s, n, _ in DENSE_D2])
def test_join_dense_delta2(shape, n_pkts, n_hosts):
    """Dense rows at delta = 2: candidates, results and the number of search-tree nodes the
    join expanded (Alg. 4-5 tuples grown through rows 1 .. r-2) match the oracle."""
    params = dict(shape, delta=2, eta=8, qp=8, rp=2, etap=64, deltap=64, theta=64,
                  anet_side=0, seed=1)
    g, o = _dense_sketch(params, n_pkts, n_hosts, seed=1)
    assert_scan_equal(g, o, 1, 64.0, f"dense delta 2 {shape}")
    assert gpu_hot(g)[1].sum() * 8 >= (1 << shape["q"])  # dense enough for the bulk rows
    _, levels = o.join_tuples(o.hot(1), levels=True)
    assert _join_nodes(g, 1, 64.0) == int(levels[1:shape["r"] - 1].sum())
    g.close()


@pytest.mark.parametrize("shape", [dict(SMALL), dict(SMALL, q=14, r=11, delta=2, qp=10, rp=8)],
                         ids=["small", "c2shape"])
def test_join_node_count_sparse(shape):
    """Sparse rows (the ordinary search): the expanded-node count is the oracle's tuple count."""
    rng = np.random.default_rng(3)
    g, o = sps.Sketch(shape), oracle.OracleSketch(shape)
    p = _rand_pkts(rng, 60000)
    g.ingest(dev_pkts(p), 1)
    o.ingest(p, 1)
    _, levels = o.join_tuples(o.hot(1), levels=True)
    assert _join_nodes(g, 1, 64.0) == int(levels[1:shape["r"] - 1].sum())
    g.close()


def test_rebase_parity():
    """The time-base shift (Sec. 3.2 recorders, u16 stamps): state equal to the oracle's after
    the rebase, scans of windows within the kept slices unchanged, ingest continuing in the
    new base."""
    rng = np.random.default_rng(12)
    g, o = sps.Sketch(SMALL), oracle.OracleSketch(SMALL)
    for s in range(1, 10):
        p = _rand_pkts(rng, 20000)
        g.ingest(dev_pkts(p), s)
        o.ingest(p, s)
    before = {k: g.scan(k, 30.0) for k in (1, 3)}
    g.rebase(6)
    assert o.rebase(6) == 0
    assert g.cur == 3
    assert_state_equal(g, o, "rebased")
    for k in (1, 3):
        assert np.array_equal(assert_scan_equal(g, o, k, 30.0, f"rebased k={k}"), before[k])
    p = _rand_pkts(rng, 20000)
    g.ingest(dev_pkts(p), 4)
    o.ingest(p, 4)
    assert_state_equal(g, o, "after the rebase")
    assert_scan_equal(g, o, 3, 30.0, "after the rebase")
    with pytest.raises(sps.SpsError) as e:
        g.rebase(5)
    assert e.value.code == sps.SPS_ESLICE


def test_rebase_crosses_slice_limit():
    """A sketch driven to slice 65534, refused slice 65535, rebased, and fed on: every scan
    equals an oracle fed the same packets numbered from slice 1."""
    rng = np.random.default_rng(13)
    g = sps.Sketch(SMALL)
    g.advance(65530)
    o = oracle.OracleSketch(SMALL)
    pk = [_rand_pkts(rng, 15000) for _ in range(8)]
    for j in range(4):                     # slices 65531 .. 65534
        g.ingest(dev_pkts(pk[j]), 65531 + j)
        o.ingest(pk[j], j + 1)
    with pytest.raises(sps.SpsError) as e:
        g.ingest(dev_pkts(pk[4]), 65535)
    assert e.value.code == sps.SPS_ESLICE
    g.rebase(65534 - 4)                    # the newest 4 slices become 1 .. 4
    assert g.cur == 4
    assert_state_equal(g, o, "rebased at the limit")
    for j in range(4, 8):                  # absolute slices 65535 .. 65538
        g.ingest(dev_pkts(pk[j]), j + 1)
        o.ingest(pk[j], j + 1)
        assert_scan_equal(g, o, 3, 30.0, f"absolute slice {65531 + j}")
