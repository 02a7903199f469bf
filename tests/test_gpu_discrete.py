"""Discrete mode (one bit per recorder: the RE and LE of Sec. 3.2 and Sec. 4) against the
stamp oracle through window equivalence: after a reset, bits set by one slice are exactly
the recorders whose stamp is that slice, and the k = 1 scan is the same."""
import numpy as np
import pytest

import oracle
from gpu_util import assert_estimates_close, dev_pkts, gpu_candidates, gpu_hot, gpu_row_live
from paper_1805_09246_amd import sps

pytestmark = pytest.mark.gpu

BASE = dict(q=12, r=6, delta=5, eta=8, qp=8, rp=3, etap=64, deltap=16, theta=64, anet_side=0,
            seed=0xC0FFEE)


def _pkts(rng, n, hosts=300):
    dst = (rng.zipf(1.3, n).astype(np.uint64) % hosts * 2654435761 + 12345).astype(np.uint32)
    src = rng.integers(0, 1 << 32, n, dtype=np.uint64).astype(np.uint32)
    return np.stack([src, dst], 1)


@pytest.mark.parametrize("shape", [dict(), dict(deltap=64), dict(etap=2048, deltap=32, qp=6, theta=16),
                                   dict(rp=1, deltap=1), dict(eta=16, theta=128)],
                         ids=["shared16", "noshare", "eta2048", "dp1", "eta16"])
def test_discrete_equals_stamps_at_k1(shape):
    params = dict(BASE, **shape)
    rng = np.random.default_rng(len(shape) + params["etap"])
    o = oracle.OracleSketch(params)
    g = sps.Sketch(dict(params, mode=sps.MODE_DISCRETE))
    assert g.nbytes < sps.sps_sketch_bytes(params)
    for s in (1, 2, 3):
        p = _pkts(rng, 40000)
        o.ingest(p, s)
        if s == 3:
            g.reset()
        if s >= 3:
            g.ingest(dev_pkts(p[:17000]), s)
            g.ingest(dev_pkts(p[17000:]), s)
    sre, slea = g.state()
    assert np.array_equal(sre, (o.sre() == 3).astype(np.uint8))
    assert np.array_equal(slea, (o.slea() == 3).astype(np.uint8))
    got = g.scan(1, 20.0)
    want, cands = o.scan(1, 20.0)
    assert np.array_equal(gpu_row_live(g), o.row_live(1))
    assert np.array_equal(gpu_hot(g), o.hot(1))
    assert np.array_equal(gpu_candidates(g), cands)
    assert np.array_equal(got["host"], want["host"]) and np.array_equal(got["live"], want["live"])
    assert np.array_equal(got["flags"], want["flags"])
    assert_estimates_close(got["estimate"], want["estimate"])


def test_discrete_merge_is_union_and_errors():
    params = dict(BASE, mode=sps.MODE_DISCRETE)
    rng = np.random.default_rng(4)
    p = _pkts(rng, 50000)
    a, b, whole = (sps.Sketch(params) for _ in range(3))
    side = rng.random(len(p)) < 0.5
    a.ingest(dev_pkts(p[side]), 1)
    b.ingest(dev_pkts(p[~side]), 1)
    whole.ingest(dev_pkts(p), 1)
    m = sps.Sketch(params)
    m.merge([a, b])
    assert np.array_equal(m.export(), whole.export())
    ex = a.export()
    c = sps.Sketch(params)
    c.import_(ex)
    assert np.array_equal(c.export(), ex)
    for bad in (lambda: a.scan(2, 10.0), lambda: a.features(dev_pkts(p[:4, :1].copy()).view(-1), 1),
                lambda: a.merge([sps.Sketch(BASE)])):
        with pytest.raises(sps.SpsError):
            bad()
