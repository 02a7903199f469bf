"""Per-row stamp histograms kept by the ingest: after every operation they equal a count of
the SLE array's cells by stamp (taken from the bit-exact dump), the scans that read them
report the oracle's row live counts, and every operation that stops the counting (merge,
import, probe replay) leaves scans on the sweep with the same results.  Sketches opt in with
row_counts = 1."""
import numpy as np
import pytest

import oracle
from gpu_util import assert_scan_equal, dev_pkts
from paper_1805_09246_amd import sps

pytestmark = pytest.mark.gpu

SMALL = dict(q=12, r=6, delta=5, eta=8, qp=8, rp=3, etap=256, deltap=256, theta=64,
             anet_side=0, seed=0xB0B, row_counts=1)


def _pkts(rng, n, hosts=400):
    dst = (rng.zipf(1.2, n).astype(np.uint64) % hosts * 2654435761 + 777).astype(np.uint32)
    src = rng.integers(0, 1 << 32, n, dtype=np.uint64).astype(np.uint32)
    return np.stack([src, dst], 1)


def hist_of(g):
    buf = sps.sps_debug_copy(g.h, 3)
    if buf.size == 0:
        return None
    return buf.view(np.uint32).reshape(g.params["rp"], 65536)


def counted(g):
    """Cells per stamp value of every SLE-array row, from the dump."""
    _, slea = g.state()
    out = np.zeros((slea.shape[0], 65536), dtype=np.uint32)
    for i in range(slea.shape[0]):
        out[i] = np.bincount(slea[i], minlength=65536)
    out[:, 0] = 0  # bin 0 (never written) is not kept
    return out


def assert_hist_exact(g, where):
    h = hist_of(g)
    assert h is not None, f"{where}: histograms not kept"
    want = counted(g)
    bad = np.argwhere(h != want)
    assert bad.size == 0, f"{where}: {len(bad)} bins differ, first {bad[:4].tolist()}"


def test_histograms_follow_the_cells_through_every_update():
    rng = np.random.default_rng(31)
    g, b = sps.Sketch(SMALL), sps.Sketch(SMALL)
    o = oracle.OracleSketch(SMALL)
    for s in range(1, 7):
        p = _pkts(rng, 60000)
        print(f"histograms: slice {s}", flush=True)
        if s % 2:
            g.ingest(dev_pkts(p), s)
        else:  # batched, together with another router
            sps.sps_ingest_batched([g.h, b.h], [dev_pkts(p), dev_pkts(_pkts(rng, 9000))], s)
        o.ingest(p, s)
        assert_hist_exact(g, f"slice {s}")
        assert_scan_equal(g, o, 3, 40.0, f"slice {s}")
    # the same slice again is idempotent: no stamp changes, no counts move
    g.ingest(dev_pkts(p), 6)
    assert_hist_exact(g, "re-ingest")
    # changes from stamps older than the block's near window (age >= 128) go straight to
    # their bins
    g.advance(300)
    o.set_slice(300)
    p = _pkts(rng, 80000)
    g.ingest(dev_pkts(p), 300)
    o.ingest(p, 300)
    assert_hist_exact(g, "slice 300")
    assert_scan_equal(g, o, 400, 40.0, "window across the gap")
    # rebase shifts the bins with the stamps
    g.rebase(250)
    o.rebase(250)
    assert_hist_exact(g, "rebase")
    assert_scan_equal(g, o, 40, 40.0, "after rebase")
    g.close()
    b.close()


def test_counting_stops_on_merge_import_and_replay_then_resumes_after_reset():
    rng = np.random.default_rng(32)
    a, b = sps.Sketch(SMALL), sps.Sketch(SMALL)
    oa, ob = oracle.OracleSketch(SMALL), oracle.OracleSketch(SMALL)
    for s in (1, 2, 3):
        pa, pb = _pkts(rng, 30000), _pkts(rng, 30000)
        a.ingest(dev_pkts(pa), s)
        b.ingest(dev_pkts(pb), s)
        oa.ingest(pa, s)
        ob.ingest(pb, s)
    a.merge([b])
    oa.merge([ob])
    assert hist_of(a) is None and hist_of(b) is not None
    plain = sps.Sketch(dict(SMALL, row_counts=0))
    assert hist_of(plain) is None
    plain.close()
    assert_scan_equal(a, oa, 3, 40.0, "merged (sweep)")
    p = _pkts(rng, 30000)  # ingest after the merge: plain stores, scans still sweep
    a.ingest(dev_pkts(p), 4)
    oa.ingest(p, 4)
    assert_scan_equal(a, oa, 3, 40.0, "merged, then ingested")
    c = sps.Sketch(SMALL)
    c.import_(b.export())
    assert hist_of(c) is None
    assert_scan_equal(c, ob, 3, 40.0, "imported (sweep)")
    cells, off = sps.sps_probe_replay_record(b.h, dev_pkts(p))
    sps.sps_probe_replay(b.h, cells, off, 3)
    assert hist_of(b) is None
    for g in (a, b, c):
        g.reset()
        assert hist_of(g) is not None and not hist_of(g).any()
    o = oracle.OracleSketch(SMALL)
    p = _pkts(rng, 50000)
    a.ingest(dev_pkts(p), 1)
    o.ingest(p, 1)
    assert_hist_exact(a, "after reset")
    assert_scan_equal(a, o, 1, 40.0, "after reset")
    for g in (a, b, c):
        g.close()


def test_autotune_keeps_histograms_exact():
    """The tuner ingests the same batch once per candidate launch shape: repeated stamps
    change nothing, so the histograms equal those of one ingest."""
    rng = np.random.default_rng(33)
    gs = [sps.Sketch(SMALL) for _ in range(3)]
    ps = [_pkts(rng, n) for n in (40000, 7000, 0)]
    sps.sps_autotune_ingest([g.h for g in gs], [dev_pkts(p) for p in ps], 1)
    one = sps.Sketch(SMALL)
    sps.sps_autotune_ingest([one.h], [dev_pkts(ps[0])], 1)
    for g in gs + [one]:
        assert_hist_exact(g, "autotuned")
        g.close()
