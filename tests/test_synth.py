"""The synthetic workloads have the stated structure (no GPU)."""
import math

import numpy as np

from synth import learned as L
from synth import make_multi_stream, make_stream, router_totals
from synth.configs import C1_RECIPE, C3_RECIPE, C3_SMALL_RECIPE


def test_c1_structure(c1_stream):
    st = c1_stream
    assert st.pkts.shape == (1 << 20, 2)
    sizes = np.diff(st.slice_off)
    assert sizes.max() - sizes.min() <= 1 and sizes.sum() == 1 << 20
    # planted host j emits ceil(c/k) distinct fresh peers per slice
    for h, m in zip(st.planted_hosts, st.planted_per_slice):
        for s in (1, 7):
            p = st.slice_pkts(s)
            peers = p[p[:, 1] == h, 0]
            assert len(peers) == m and len(np.unique(peers)) == m
    # deterministic
    again = make_stream(C1_RECIPE)
    assert np.array_equal(again.pkts, st.pkts)


def test_multi_router_structure():
    t = router_totals(C3_RECIPE)
    assert len(t) == 16 and np.median(t) > 2 ** 20
    rs = make_multi_stream(C3_SMALL_RECIPE)
    assert len(rs) == 16
    # a planted host's peers of one slice are split over routers and never repeated
    h = rs[0].planted_hosts[0]
    per = [r.slice_pkts(3) for r in rs]
    peers = np.concatenate([p[p[:, 1] == h, 0] for p in per])
    assert len(peers) == rs[0].planted_per_slice[0] == len(np.unique(peers))
    assert sum((p[:, 1] == h).any() for p in per) > 8


def test_learned_generator_last_slice_law():
    """Last appearance: first slice uniform on 1..10, each later slice w.p. 0.3, so
    P(last = s) = sum_{f<=s} 1/10 * (0.7^(10-f) if s == f else 0.3 * 0.7^(10-s))."""
    cards = np.array([40000, 25000, 35000], dtype=np.int64)
    hosts = L.host_addrs(0, 3)
    b = L.planted_cpu(hosts, cards, L.peer_salts(1, 3), key=99)
    n = np.array([len(x) for x in b], dtype=np.float64)
    assert n.sum() == cards.sum()
    for s in range(1, 11):
        p = sum(0.1 * (0.7 ** (10 - f) if s == f else 0.3 * 0.7 ** (10 - s))
                for f in range(1, s + 1))
        assert abs(n[s - 1] / n.sum() - p) < 5 * math.sqrt(p * (1 - p) / n.sum())
    # peers of one host are distinct
    allp = np.concatenate(b)
    for h in hosts:
        peers = allp[allp[:, 1] == h, 0]
        assert len(peers) == len(np.unique(peers))


def test_learned_cards_log_uniform():
    c = L.draw_cards(7, 200000)
    assert c.min() >= 1 and c.max() <= 1e6
    frac = np.mean(np.log(c) < math.log(1e3))
    assert abs(frac - 0.5) < 0.01
