"""Pins of the CPU oracle against what the paper and the mathematics fix (no GPU).

Every check here compares the oracle with something other than itself: values printed in
the paper (tests/golden/paper_values.json), published test vectors of the hash primitives,
closed forms (Eq. 1, Eq. 2-5, Eq. 8-12), exhaustive search, and invariants of the stamp
representation (window equivalence, merge union, order independence).
"""
import math
from fractions import Fraction

import numpy as np
import pytest

import oracle
from oracle import truth
from conftest import golden

M32 = (1 << 32) - 1
M64 = (1 << 64) - 1


# ---------------------------------------------------------------- paper's worked values
def test_lsb_paper_examples():
    g = golden("paper_values.json")["lsb_examples"]
    for v, want in g["cases"]:
        assert oracle.lsb(v) == want
    # reading: LSB(0) = 32, so exactly the h with their low tau bits clear are sampled
    assert oracle.lsb(0) == 32
    assert oracle.lsb(1 << 31) == 31


def test_tau_eq1():
    for theta, eta, want in golden("paper_values.json")["tau_examples"]["cases"]:
        assert oracle.tau(theta, eta) == want
        assert want == max(0, math.ceil(math.log2(theta / eta)))


def test_hot_cut_rho():
    g = golden("paper_values.json")["rho"]
    rho = 0.99 * (1.0 - math.exp(-1.0 / 3.0))
    assert abs(rho * g["eta"] - g["rho_times_eta"]) < 1e-6
    assert oracle.hot_cut(g["eta"]) == g["integer_cut"]
    assert oracle.hot_cut(16) == math.ceil(16 * rho) == 5


def test_paper_memory_and_mrr():
    p = golden("paper_values.json")["paper_parameters"]
    m = golden("paper_values.json")["paper_memory"]
    params = dict(q=p["q"], r=p["r"], delta=p["delta"], eta=p["eta"], qp=p["qp"], rp=p["rp"],
                  etap=p["etap"], deltap=p["deltap"], theta=p["theta"], anet_side=0, seed=1)
    # the paper's own parameters violate the RHFG coverage condition: (5-2)*5+17 = 32 holds
    sk = oracle.OracleSketch(params)
    assert sk.row_len == m["slea_row_len"]
    assert sk.sre().nbytes == m["sre_bytes"]
    assert sk.slea().nbytes == m["slea_bytes"]
    assert abs(oracle.mrr(p["qp"], p["etap"], p["deltap"]) - m["mrr"]) < 1e-15
    # no sharing (delta' = eta') saves nothing
    assert oracle.mrr(p["qp"], p["etap"], p["etap"]) == 0.0


# ---------------------------------------------------------------- hash primitives and spec
def test_fmix32_vectors():
    for x, want in golden("hash_vectors.json")["murmur3_fmix32"]["cases"]:
        assert oracle.fmix32(x) == want


def test_splitmix64_vectors():
    g = golden("hash_vectors.json")["splitmix64"]
    st = 1234567
    for want in g["seed_1234567"]:
        assert oracle.splitmix64_next(st) == int(want)
        st = (st + 0x9E3779B97F4A7C15) & M64
    assert oracle.splitmix64_next(0) == int(g["seed_0_first"])


def _spec_hashes(params):
    """The hash specification, restated: seed j is the low 32 bits of the (j+1)-th SplitMix64
    output from params.seed; h_j(x) = fmix32(x xor seed_j), reduced by a power-of-two mask."""
    st, seeds = params["seed"], []
    for _ in range(4 + params["rp"]):
        seeds.append(oracle.splitmix64_next(st) & M32)
        st = (st + 0x9E3779B97F4A7C15) & M64
    f = oracle.fmix32
    q, qp = params["q"], params["qp"]
    return dict(
        H1=lambda x: f(x ^ seeds[0]),
        H2=lambda x: f(x ^ seeds[1]) & (params["eta"] - 1),
        H3=lambda x: f(x ^ seeds[2]) & (params["etap"] - 1),
        RHFG0=lambda x: f(x ^ seeds[3]) & ((1 << q) - 1),
        LH=lambda i, x: f(x ^ seeds[4 + i]) & ((1 << qp) - 1),
    )


def test_hash_spec_composition():
    from synth.configs import C1_PARAMS, C2_PARAMS
    rng = np.random.default_rng(7)
    for params in (C1_PARAMS, C2_PARAMS):
        sk = oracle.OracleSketch(params)
        h = _spec_hashes(params)
        for x in [0, 1, M32, 0x80000000] + [int(v) for v in rng.integers(0, 1 << 32, 200)]:
            assert sk.hash(sk.H1, 0, x) == h["H1"](x)
            assert sk.hash(sk.H2, 0, x) == h["H2"](x)
            assert sk.hash(sk.H3, 0, x) == h["H3"](x)
            assert sk.hash(sk.RHFG, 0, x) == h["RHFG0"](x)
            for i in range(params["rp"]):
                assert sk.hash(sk.LH, i, x) == h["LH"](i, x)


def test_rhfg_eq7_recovers_address_bits():
    """Eq. 7: RHFG[i](x) xor RHFG[0](x) gives the q address bits at shift (i-1)*delta, and
    together rows 1..r-1 cover all 32 bits (coverage (r-2)*delta + q >= 32)."""
    from synth.configs import C1_PARAMS, C2_PARAMS
    rng = np.random.default_rng(3)
    for params in (C1_PARAMS, C2_PARAMS):
        sk = oracle.OracleSketch(params)
        q, d, r = params["q"], params["delta"], params["r"]
        for x in [0, M32, 1, 1 << 31] + [int(v) for v in rng.integers(0, 1 << 32, 300)]:
            c0 = sk.hash(sk.RHFG, 0, x)
            y = 0
            for i in range(1, r):
                B = sk.hash(sk.RHFG, i, x) ^ c0
                assert B == (x >> ((i - 1) * d)) & ((1 << q) - 1)
                y |= B << ((i - 1) * d)
            assert y == x


def test_sampling_rate_is_two_to_minus_tau():
    """H1 is a bijection, so LSB(H1(bip)) >= tau for a 2^-tau share of addresses."""
    from synth.configs import C1_PARAMS
    sk = oracle.OracleSketch(C1_PARAMS)
    rng = np.random.default_rng(11)
    xs = rng.integers(0, 1 << 32, 20000)
    hits = sum(1 for x in xs if oracle.lsb(sk.hash(sk.H1, 0, int(x))) >= 3)
    p = 2.0 ** -3
    assert abs(hits / len(xs) - p) < 5 * math.sqrt(p * (1 - p) / len(xs))


# ---------------------------------------------------------------- candidate recovery
JOIN_PARAMS = [
    dict(q=12, r=6, delta=5),   # coverage exactly 32
    dict(q=10, r=7, delta=5),   # 35 bits: top rows must reject bits above 31
    dict(q=14, r=11, delta=2),  # config-2 shape
    dict(q=8, r=11, delta=3),   # 35 bits, narrow columns
]


@pytest.mark.parametrize("shape", JOIN_PARAMS)
def test_join_tuples_equals_exhaustive(shape):
    """The paper's tuple growing (Alg. 4-5) and the plain definition agree exactly."""
    params = dict(shape, eta=8, qp=4, rp=1, etap=16, deltap=16, theta=1024, anet_side=0,
                  seed=0xABCDEF + shape["q"])
    sk = oracle.OracleSketch(params)
    rng = np.random.default_rng(shape["q"] * 31 + shape["r"])
    ncol = 1 << shape["q"]
    # random hot cells plus the columns of some chosen addresses (so real hits exist)
    density = {12: 0.04, 10: 0.05, 14: 0.04, 8: 0.05}[shape["q"]]
    hot = (rng.random((shape["r"], ncol)) < density).astype(np.uint8)
    chosen = [int(v) for v in rng.integers(0, 1 << 32, 25)]
    for x in chosen:
        for i in range(shape["r"]):
            hot[i, sk.hash(sk.RHFG, i, x)] = 1
    got_b = sk.join_brute(hot)
    got_t = sk.join_tuples(hot)
    assert np.array_equal(got_b, got_t)
    assert set(chosen) <= set(got_b.tolist())
    for x in got_b[:200]:
        assert all(hot[i, sk.hash(sk.RHFG, i, int(x))] for i in range(shape["r"]))


def test_join_empty_and_full_rows():
    params = dict(q=12, r=6, delta=5, eta=8, qp=4, rp=1, etap=16, deltap=16, theta=1024,
                  anet_side=0, seed=5)
    sk = oracle.OracleSketch(params)
    hot = np.zeros((6, 4096), np.uint8)
    assert len(sk.join_tuples(hot)) == 0
    hot[:, :] = 1
    hot[0, :] = 0
    hot[0, 17] = 1
    # every address whose RHFG[0] is 17: 2^32 / 2^12 of them (too many partial tuples for
    # the tuple-growing form, so the exhaustive form is checked here)
    got = sk.join_brute(hot, cap=1 << 21)
    assert len(got) == 1 << 20
    assert all(sk.hash(sk.RHFG, 0, int(x)) == 17 for x in got[::4096])


@pytest.mark.parametrize("shape", [dict(q=6, r=15, delta=2), dict(q=8, r=10, delta=3)])
def test_join_tuple_levels_count_prefixes(shape):
    """The tuples grown through row i are the pairs (he0, x) of a hot row-0 column and an
    address prefix of (i - 1) delta + q bits whose windows B(1..i) (Eq. 7) land on hot columns
    he0 ^ B(j) of rows 1..i.  Counted here by enumerating every prefix, for the rows whose
    prefixes have at most 20 bits, on dense random rows."""
    q, r, d = shape["q"], shape["r"], shape["delta"]
    params = dict(shape, eta=8, qp=4, rp=1, etap=16, deltap=16, theta=1024, anet_side=0, seed=9)
    sk = oracle.OracleSketch(params)
    rng = np.random.default_rng(q * 7 + r)
    hot = (rng.random((r, 1 << q)) < 0.3).astype(np.uint8)
    _, levels = sk.join_tuples(hot, levels=True)
    he0 = np.nonzero(hot[0])[0].astype(np.int64)
    qm = (1 << q) - 1
    checked = 0
    for i in range(1, r):
        bits = (i - 1) * d + q
        if bits > 20:
            break
        x = np.arange(1 << bits, dtype=np.int64)
        ok = np.ones((len(he0), len(x)), dtype=bool)
        for j in range(1, i + 1):
            win = (x >> ((j - 1) * d)) & qm
            ok &= hot[j][he0[:, None] ^ win[None, :]].astype(bool)
        assert int(levels[i]) == int(ok.sum()), f"row {i}"
        checked += 1
    assert checked >= 3
    assert levels[1] == hot[0].sum() * hot[1].sum()


# ---------------------------------------------------------------- estimator laws
def _surjections(alpha, eta):
    """Lemma (Sec. 3.2, full version): FN(alpha, eta) = eta^alpha - sum_{i<eta} C(eta,i) FN(alpha,i),
    FN(alpha, 1) = 1 -- the number of ways alpha balls fill all eta boxes."""
    fn = {1: 1}
    for j in range(2, eta + 1):
        fn[j] = j ** alpha - sum(math.comb(j, i) * fn[i] for i in range(1, j))
    return fn


def _p_weight(card, eta, tau, amax=120):
    """Eq. 3-5: P(weight = eta1) for an isolated host with `card` distinct peers."""
    p = Fraction(1, 2 ** tau)
    out = [Fraction(0)] * (eta + 1)
    for alpha in range(0, min(card, amax) + 1):
        pa = math.comb(card, alpha) * p ** alpha * (1 - p) ** (card - alpha)   # Eq. 4
        if alpha == 0:
            out[0] += pa
            continue
        fn = _surjections(alpha, eta)
        for e1 in range(1, min(alpha, eta) + 1):
            out[e1] += pa * Fraction(math.comb(eta, e1) * fn[e1], eta ** alpha)   # Eq. 2-3
    return [float(v) for v in out]


def test_sre_fill_law_eq5():
    """Histogram of SRE weights of isolated hosts against Eq. 2-5 (chi-square)."""
    card, nh = 512, 3000
    params = dict(q=16, r=6, delta=4, eta=8, qp=4, rp=1, etap=16, deltap=16, theta=1024,
                  anet_side=0, seed=0x1234)
    sk = oracle.OracleSketch(params)
    rng = np.random.default_rng(21)
    hosts = rng.choice(1 << 32, size=nh, replace=False).astype(np.uint32)
    cols = np.array([sk.hash(sk.RHFG, 0, int(h)) for h in hosts])
    uniq, cnt = np.unique(cols, return_counts=True)
    alone = np.isin(cols, uniq[cnt == 1])
    peers = rng.choice(1 << 32, size=(nh, card), replace=False).astype(np.uint32)
    pk = np.stack([peers.ravel(), np.repeat(hosts, card)], 1)
    assert sk.ingest(pk, 1) == 0
    w = (sk.sre()[0, cols[alone]] >= 1).sum(1)
    tau = sk.tau
    probs = _p_weight(card, 8, tau)
    assert abs(sum(probs) - 1) < 1e-9
    n = int(alone.sum())
    obs = np.bincount(w, minlength=9)
    # pool the sparse tail bins
    exp = np.array(probs) * n
    bins_o, bins_e, acc_o, acc_e = [], [], 0, 0.0
    for o, e in zip(obs, exp):
        acc_o += o
        acc_e += e
        if acc_e >= 20:
            bins_o.append(acc_o)
            bins_e.append(acc_e)
            acc_o, acc_e = 0, 0.0
    bins_o[-1] += acc_o
    bins_e[-1] += acc_e
    chi2 = sum((o - e) ** 2 / e for o, e in zip(bins_o, bins_e))
    dof = len(bins_o) - 1
    assert chi2 < dof + 6 * math.sqrt(2 * dof), (chi2, dof, obs, exp)
    # P(hot | 512) from Eq. 5
    p_hot = sum(probs[3:])
    assert abs(p_hot - 0.672) < 0.01
    assert abs((w >= 3).mean() - p_hot) < 5 * math.sqrt(p_hot * (1 - p_hot) / n)


def test_linear_counting_zero_cells():
    """Empty SLE cells after n distinct peers: E[Z] = m(1-1/m)^n and its variance (Whang et al.)."""
    m, n, nh = 1024, 1000, 1500
    params = dict(q=12, r=6, delta=5, eta=8, qp=13, rp=1, etap=m, deltap=m, theta=1024,
                  anet_side=0, seed=0x77)
    sk = oracle.OracleSketch(params)
    rng = np.random.default_rng(5)
    hosts = rng.choice(1 << 32, size=nh, replace=False).astype(np.uint32)
    sle = np.array([sk.hash(sk.LH, 0, int(h)) for h in hosts])
    uniq, cnt = np.unique(sle, return_counts=True)
    alone = np.isin(sle, uniq[cnt == 1])
    peers = rng.choice(1 << 32, size=(nh, n), replace=False).astype(np.uint32)
    sk.ingest(np.stack([peers.ravel(), np.repeat(hosts, n)], 1), 1)
    rows = sk.slea()[0].reshape(1 << 13, m)
    Z = (rows[sle[alone]] == 0).sum(1).astype(np.float64)
    EZ = m * (1 - 1 / m) ** n
    VZ = m * (m - 1) * (1 - 2 / m) ** n + m * (1 - 1 / m) ** n - m * m * (1 - 1 / m) ** (2 * n)
    k = len(Z)
    assert abs(Z.mean() - EZ) < 4 * math.sqrt(VZ / k), (Z.mean(), EZ)
    assert 0.75 < Z.var() / VZ < 1.3


def test_eq9_and_eq12():
    params = dict(q=12, r=6, delta=5, eta=8, qp=4, rp=3, etap=1024, deltap=1024, theta=1024,
                  anet_side=0, seed=1)
    sk = oracle.OracleSketch(params)
    L = sk.row_len
    # no other host in the SLE array (SF = 0): Eq. 12 leaves U unchanged, Eq. 9 applies
    for U in (0, 1, 100, 512, 1000, 1023):
        est, fl = sk.estimate_one(U, np.zeros(3, np.uint64), 1e9)
        assert abs(est - (-1024 * math.log((1024 - U) / 1024))) <= 1e-12 * max(1, est)
        assert fl == 0
    # full union SLE saturates: clamped to eta' - 1
    est, fl = sk.estimate_one(1024, np.zeros(3, np.uint64), 1e9)
    assert fl & oracle.F_SATURATED and abs(est - 1024 * math.log(1024)) < 1e-9
    # Eq. 11 holds for the corrected weight: U = w + (eta' - w) * prod SF
    rl = np.array([L // 4, L // 3, L // 2], np.uint64)
    P = (rl[0] / L) * (rl[1] / L) * (rl[2] / L)
    for U in (100, 300, 700):
        est, _ = sk.estimate_one(U, rl, 1e9)
        w = 1024 * (1 - math.exp(-est / 1024))
        assert abs(U - (w + (1024 - w) * P)) < 1e-9 * U
    # fewer live cells than the noise expectation: clamped to 0
    est, fl = sk.estimate_one(10, rl, 1e9)
    assert est == 0.0 and fl & oracle.F_CLAMPLOW


# ---------------------------------------------------------------- stamp-sketch invariants
SMALL = dict(q=12, r=6, delta=5, eta=8, qp=8, rp=3, etap=64, deltap=16, theta=64, anet_side=0,
             seed=0xC0FFEE)


def _small_stream(seed, n_slices=8, per=3000, hosts=300):
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(n_slices):
        dst = rng.zipf(1.3, per).astype(np.uint64) % hosts
        dst = (dst * 2654435761 + 12345).astype(np.uint32)
        src = rng.integers(0, 1 << 32, per, dtype=np.uint64).astype(np.uint32)
        out.append(np.stack([src, dst], 1))
    return out


def test_window_equivalence():
    """Cells live at (cur, k) are exactly the cells a fresh sketch fed only the window's
    slices has written (Sec. 3.2: a recorder is within the window iff its distance < k)."""
    sl = _small_stream(1)
    for k in (1, 3, 5):
        full = oracle.OracleSketch(SMALL)
        for s, p in enumerate(sl, 1):
            full.ingest(p, s)
        cur = len(sl)
        win = oracle.OracleSketch(SMALL)
        for s in range(cur - k + 1, cur + 1):
            win.ingest(sl[s - 1], s)
        lo = cur - k + 1
        assert np.array_equal(full.sre() >= lo, win.sre() > 0)
        assert np.array_equal(full.slea() >= lo, win.slea() > 0)
        assert np.array_equal(full.hot(k), win.hot(k))
        assert np.array_equal(full.row_live(k), win.row_live(k))


@pytest.mark.parametrize("deltap", [16, 64])
def test_features_window_equivalence(deltap):
    """Per-age features of the learned estimator: x_a after slice cur counts the union-SLE
    cells of a host that a fresh sketch fed only slices cur-a .. cur has written in every row
    (Alg. 8 union over the window of the newest a+1 slices), for every a < k.  The fresh
    sketch's count is taken from its raw cells here, not from the features routine."""
    params = dict(SMALL, deltap=deltap)
    sl = _small_stream(6, n_slices=9)
    cur, k = len(sl), 7
    full = oracle.OracleSketch(params)
    for s, p in enumerate(sl, 1):
        full.ingest(p, s)
    h = _spec_hashes(params)
    rng = np.random.default_rng(2)
    hosts = np.concatenate([np.unique(sl[-1][:, 1])[:40],
                            rng.integers(0, 1 << 32, 10, dtype=np.uint64).astype(np.uint32)])
    x = full.features(k, hosts)
    assert np.all(np.diff(x.astype(np.int64), axis=1) >= 0)  # older ages only add cells
    for a in range(k):
        fresh = oracle.OracleSketch(params)
        for s in range(cur - a, cur + 1):
            fresh.ingest(sl[s - 1], s)
        written = fresh.slea() > 0
        for j, hh in enumerate(hosts.tolist()):
            m = np.ones(params["etap"], bool)
            for i in range(params["rp"]):
                j0 = h["LH"](i, hh) * deltap
                m &= written[i, j0:j0 + params["etap"]]
            assert x[j, a] == int(m.sum()), (a, hh)


def test_features_from_packets():
    """The same counts straight from the packets, with no sketch at all: with delta' = eta'
    (no shared cells) cell z of host x's union SLE is set over a window exactly when, in every
    row i, some packet of the window has LH_i(aip) = LH_i(x) and H3(bip) = z (Alg. 6, Alg. 8)."""
    params = dict(SMALL, deltap=64, qp=6)
    sl = _small_stream(7, n_slices=6, per=400, hosts=60)
    cur, k = len(sl), 4
    sk = oracle.OracleSketch(params)
    for s, p in enumerate(sl, 1):
        sk.ingest(p, s)
    h = _spec_hashes(params)
    hosts = np.unique(np.concatenate(sl)[:, 1])[:25]
    x = sk.features(k, hosts)
    for a in range(k):
        win = np.concatenate(sl[cur - a - 1:])
        for j, hh in enumerate(hosts.tolist()):
            sets = []
            for i in range(params["rp"]):
                li = h["LH"](i, hh)
                sets.append({h["H3"](src) for src, dst in win.tolist() if h["LH"](i, dst) == li})
            assert x[j, a] == len(set.intersection(*sets)), (a, hh)


def test_k1_is_discrete_re_le():
    """k = 1 (discrete window): live cells are those set in the current slice alone."""
    sl = _small_stream(2, n_slices=3)
    a = oracle.OracleSketch(SMALL)
    for s, p in enumerate(sl, 1):
        a.ingest(p, s)
    b = oracle.OracleSketch(SMALL)
    b.ingest(sl[-1], 3)
    assert np.array_equal(a.slea() == 3, b.slea() > 0)
    assert np.array_equal(a.hot(1), b.hot(1))


def test_merge_union():
    """Sketch of the union of two routers' packets == cell-wise max of their sketches."""
    sl = _small_stream(3)
    rng = np.random.default_rng(9)
    whole, ra, rb = (oracle.OracleSketch(SMALL) for _ in range(3))
    for s, p in enumerate(sl, 1):
        side = rng.random(len(p)) < 0.4
        whole.ingest(p, s)
        ra.ingest(p[side], s)
        rb.ingest(p[~side], s)
    merged = oracle.OracleSketch(SMALL)
    assert merged.merge([ra, rb]) == 0
    assert np.array_equal(merged.sre(), whole.sre())
    assert np.array_equal(merged.slea(), whole.slea())
    assert merged.cur == whole.cur
    # a single router alone misses cells
    assert not np.array_equal(ra.slea(), whole.slea())
    other = dict(SMALL, seed=SMALL["seed"] + 1)
    assert merged.merge([oracle.OracleSketch(other)]) == -3


def test_threaded_ingest_equals_plain_ingest(c1_stream):
    """Splitting the ingest's rows over threads writes the same cells (any thread count)."""
    from synth.configs import C1_PARAMS
    a = oracle.OracleSketch(C1_PARAMS)
    for s in (1, 2, 3):
        a.ingest(c1_stream.slice_pkts(s), s)
    for threads in (1, 3, 16):
        b = oracle.OracleSketch(C1_PARAMS)
        for s in (1, 2, 3):
            assert b.ingest_threads(c1_stream.slice_pkts(s), s, threads) == 0
        assert np.array_equal(a.sre(), b.sre()) and np.array_equal(a.slea(), b.slea())
        assert b.cur == 3
    assert oracle.OracleSketch(C1_PARAMS).ingest_threads(c1_stream.slice_pkts(1), 0) != 0


def test_order_independence():
    sl = _small_stream(4)
    a, b = oracle.OracleSketch(SMALL), oracle.OracleSketch(SMALL)
    rng = np.random.default_rng(0)
    for s, p in enumerate(sl, 1):
        a.ingest(p, s)
        q = p[rng.permutation(len(p))]
        b.ingest(q[: len(q) // 2], s)
        b.ingest(q[len(q) // 2:], s)
    assert np.array_equal(a.sre(), b.sre()) and np.array_equal(a.slea(), b.slea())


def test_rebase_equals_relabelled_stream():
    """Rebasing the sketch of slices 1..n by `off` gives exactly the sketch of slices off+1..n
    alone, relabelled s - off: cells last written at or before slice off read as never
    written (0), the others keep their age (Sec. 3.2: only the distance matters)."""
    sl = _small_stream(8, n_slices=9)
    for off in (0, 3, 8, 9):
        full = oracle.OracleSketch(SMALL)
        for s, p in enumerate(sl, 1):
            full.ingest(p, s)
        assert full.rebase(off) == 0 and full.cur == 9 - off
        fresh = oracle.OracleSketch(SMALL)
        for s in range(off + 1, 10):
            fresh.ingest(sl[s - 1], s - off)
        assert np.array_equal(full.sre(), fresh.sre())
        assert np.array_equal(full.slea(), fresh.slea())
    assert full.rebase(1) == -2  # below slice 0


def test_rebase_keeps_short_windows():
    """Scans of any window k <= cur - offset give the same hot SREs, row counts, features and
    report after the rebase; a longer window loses the slices shifted out."""
    sl = _small_stream(9, n_slices=10)
    a, b = oracle.OracleSketch(SMALL), oracle.OracleSketch(SMALL)
    for s, p in enumerate(sl, 1):
        a.ingest(p, s)
        b.ingest(p, s)
    assert b.rebase(6) == 0 and b.cur == 4
    hosts = np.unique(sl[-1][:, 1])[:30]
    for k in (1, 2, 4):
        assert np.array_equal(a.hot(k), b.hot(k))
        assert np.array_equal(a.row_live(k), b.row_live(k))
        assert np.array_equal(a.features(k, hosts), b.features(k, hosts))
        ra, _ = a.scan(k, 20.0)
        rb, _ = b.scan(k, 20.0)
        assert np.array_equal(ra, rb)
    assert (a.row_live(8) > b.row_live(8)).all()
    # ingest continues in the new time base
    p = _small_stream(10, n_slices=1)[0]
    a.ingest(p, 11)
    b.ingest(p, 5)
    assert np.array_equal(a.scan(3, 20.0)[0], b.scan(3, 20.0)[0])


def test_slice_rules():
    sk = oracle.OracleSketch(SMALL)
    p = _small_stream(5, n_slices=1)[0]
    assert sk.ingest(p, 0) == -2
    assert sk.ingest(p, 3) == 0
    assert sk.ingest(p, 2) == -2
    assert sk.ingest(p, 3) == 0
    assert sk.ingest(p, 65535) == -2
    assert sk.ingest(p, 65534) == 0


def test_tiny_sle_by_enumeration():
    """Shared-cell SLE array (delta' < eta', Sec. 4): every cell checked against a plain
    enumeration of the pairs, with the per-pair cells written out by hand."""
    params = dict(q=12, r=6, delta=5, eta=8, qp=4, rp=2, etap=16, deltap=4, theta=1024,
                  anet_side=0, seed=99)
    sk = oracle.OracleSketch(params)
    h = _spec_hashes(params)
    assert sk.row_len == 16 * 4 + 16 - 4
    rng = np.random.default_rng(1)
    expect = np.zeros((2, sk.row_len), np.uint16)
    for s in (1, 2, 4):
        pk = rng.integers(0, 1 << 32, size=(150, 2), dtype=np.uint64).astype(np.uint32)
        pk[:, 1] = pk[:, 1] % 7   # few hosts
        sk.ingest(pk, s)
        for src, dst in pk.tolist():
            for i in range(2):
                expect[i, h["LH"](i, dst) * 4 + h["H3"](src)] = s
    assert np.array_equal(sk.slea(), expect)


# ---------------------------------------------------------------- scan pieces vs numpy
def test_scan_pieces_against_numpy(c1_oracle):
    sk = c1_oracle
    p = sk.params
    k, cur = 5, sk.cur
    lo = cur - k + 1
    assert np.array_equal(sk.row_live(k), (sk.slea() >= lo).sum(1).astype(np.uint64))
    assert np.array_equal(sk.hot(k), ((sk.sre() >= lo).sum(2) >= 3).astype(np.uint8))
    hosts = np.array([12345, 0xDEADBEEF, 7], np.uint32)
    x = sk.features(k, hosts)
    slea = sk.slea()
    for j, hh in enumerate(hosts.tolist()):
        m = np.min([slea[i, sk.hash(sk.LH, i, hh) * p["deltap"]:][: p["etap"]]
                    for i in range(p["rp"])], axis=0)
        for a in range(k):
            assert x[j, a] == int((m >= max(1, cur - a)).sum())


def test_exact_truth_bruteforce():
    from synth import Stream, StreamRecipe
    rng = np.random.default_rng(8)
    pk = rng.integers(0, 50, size=(4000, 2)).astype(np.uint32)
    off = np.array([0, 1000, 2000, 3000, 4000])
    st = Stream(StreamRecipe("t", 0, 4000, 4, 2, 1, 1.0, []), pk, off, np.zeros(0, np.uint32),
                np.zeros(0, np.int64))
    hosts, counts = truth.cardinalities(truth.window_pairs(st, 4, 2))
    want = {}
    for src, dst in pk[2000:4000].tolist():
        want.setdefault(dst, set()).add(src)
    assert dict(zip(hosts.tolist(), counts.tolist())) == {h: len(v) for h, v in want.items()}
    fpr, fnr, tfr = truth.detection_rates([1, 2, 3, 4], [2, 3, 9])
    assert (fpr, fnr, tfr) == (0.25, 0.5, 0.75)


def test_sliding_truth_equals_python_sets_per_window():
    """The all-windows exact truth (each pair's occurrences cover a range of window ends)
    equals Def. 1-2 evaluated window by window with python sets, for every window end and
    several window lengths, on a stream with repeated pairs, gaps and a host below theta."""
    from synth import Stream, StreamRecipe
    rng = np.random.default_rng(9)
    n_sl, per = 9, 700
    pk = rng.integers(0, 40, size=(n_sl * per, 2)).astype(np.uint32)
    pk[:, 1] %= 6  # six hosts, many repeated pairs
    pk[pk[:, 1] == 5, 0] %= 3  # host 5 has three peers only: dropped at theta_min 4
    off = np.arange(0, n_sl * per + 1, per)
    st = Stream(StreamRecipe("t", 0, n_sl * per, n_sl, 3, 1, 1.0, []), pk, off,
                np.zeros(0, np.uint32), np.zeros(0, np.int64))
    card = truth.sliding_cardinalities(st, [1, 2, 4, 12], 4)
    assert 5 not in card[1][0].tolist()
    for k in (1, 2, 4, 12):
        hosts, counts = card[k]
        for cur in range(1, n_sl + 1):
            want = {}
            for src, dst in pk[off[max(1, cur - k + 1) - 1]:off[cur]].tolist():
                want.setdefault(dst, set()).add(src)
            got = dict(zip(hosts.tolist(), counts[:, cur - 1].tolist()))
            assert got == {h: len(v) for h, v in want.items() if h != 5}, (k, cur)
            th, tc = truth.sliding_super_points(card, k, cur, 30)
            assert th.tolist() == sorted(h for h, v in want.items() if len(v) >= 30)


def test_c1_scan_reports_planted(c1_oracle, c1_stream):
    """Every planted host is reported; unsaturated estimates are near the truth."""
    res, cands = c1_oracle.scan(5, 1024.0)
    assert np.all(np.diff(res["host"].astype(np.int64)) > 0)
    assert np.all(np.diff(cands.astype(np.int64)) > 0)
    rep = dict(zip(res["host"].tolist(), res["estimate"].tolist()))
    hosts, counts = truth.cardinalities(truth.window_pairs(c1_stream, 10, 5))
    true = dict(zip(hosts.tolist(), counts.tolist()))
    for h in c1_stream.planted_hosts.tolist():
        assert h in rep
        if true[h] < 5000:
            assert abs(rep[h] - true[h]) / true[h] < 0.2
    th, _ = truth.super_points(c1_stream, 10, 5, 1024)
    fpr, fnr, _ = truth.detection_rates(th, res["host"])
    assert fnr < 0.2 and fpr < 0.5


# ---------------------------------------------------------------- learned estimator oracle
def test_mlp_gradient_finite_differences():
    from oracle import mlp
    p = mlp.init_params(3)
    rng = np.random.default_rng(0)
    x = rng.random((16, 10))
    t = rng.random(16) * 5
    loss, g = mlp.loss_and_grad(p, x, t)
    v = mlp.flatten(p)
    gv = mlp.flatten(g)
    assert v.size == mlp.N_PARAMS == 4929
    idx = rng.choice(v.size, 60, replace=False)
    for i in idx:
        e = np.zeros_like(v)
        e[i] = 1e-6
        lp, _ = mlp.loss_and_grad(mlp.unflatten(v + e), x, t)
        lm, _ = mlp.loss_and_grad(mlp.unflatten(v - e), x, t)
        fd = (lp - lm) / 2e-6
        assert abs(fd - gv[i]) <= 1e-6 + 1e-5 * abs(fd)


def test_adam_first_step_moves_by_lr():
    """At step 1 bias correction makes the Adam update -lr * g / (|g| + eps)."""
    from oracle import mlp
    p = mlp.init_params(1)
    g = {n: np.full(s, 0.5) for n, s in mlp.SHAPES}
    z = {n: np.zeros(s) for n, s in mlp.SHAPES}
    p1, m1, v1 = mlp.adam_step(p, g, z, z, 1, lr=1e-2)
    for n, _ in mlp.SHAPES:
        assert np.allclose(p1[n] - p[n], -1e-2 * 0.5 / (0.5 + 1e-8), rtol=0, atol=1e-15)
        assert np.allclose(m1[n], 0.05) and np.allclose(v1[n], 0.00025)
