"""Learned cardinality estimator: data through the sketch, training with the library's kernels,
gating, and evaluation against linear counting.

The paper estimates a candidate's cardinality by linear counting over its union SLE (Alg. 8,
Eq. 9, Eq. 12).  Linear counting only sees the window-wide live count |USLE|^k and
saturates near eta' ln eta' (7,098 for eta' = 1024).  The learned estimator reads the live
counts at every window age (x_a for a < 10: cells last written within the newest a+1
slices); younger ages stay unsaturated longer, which is where it can beat linear counting.
Linear counting remains the fallback and the judge of its error.

Every compute step runs in libsps.so: features (sps_features), estimates (sps_estimate_hosts),
gradients (sps_mlp_grad), Adam (sps_mlp_adam), inference (sps_mlp_forward and inside scans).
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np
import torch

from . import sps

WINDOW = 10
DECADES = [(1, 10), (10, 100), (100, 1_000), (1_000, 10_000), (10_000, 100_000),
           (100_000, 1_000_001)]


@dataclasses.dataclass
class Dataset:
    features: np.ndarray   # (n, 10) uint32 per-age live counts
    cards: np.ndarray      # (n,) true cardinalities
    lc: np.ndarray         # (n,) linear-counting estimates (sketch path, no network)
    lc_flags: np.ndarray   # (n,) flags of those estimates
    etap: int


def make_backgrounds(params: dict, seed: int, n: int = 4) -> list:
    """Sketches of n background streams (one window each) to embed hosts into."""
    from synth import make_stream
    from synth import learned as L
    bases = []
    for b in range(n):
        st = make_stream(L.background_recipe(seed * 131 + b))
        sk = sps.Sketch(params)
        for s in range(1, WINDOW + 1):
            sk.ingest(torch.from_numpy(st.slice_pkts(s).view(np.int32)).cuda(), s)
        bases.append(sk)
    return bases


def generate(params: dict, n_hosts: int, seed: int, bases: list | None = None,
             hosts_per_stream: int = 150, peer_budget: int = 16_000_000, log=None,
             law: int = 0) -> Dataset:
    """Hosts with log-uniform cardinalities embedded into background streams, ingested by the
    GPU sketch; per-age features and linear-counting estimates read back per host.  law: the
    peers' arrival over the window (0: the training law; 1: fresh peers spread evenly over
    the slices, as the scale workload's planted hosts)."""
    from synth import learned as L

    cards = L.draw_cards(seed, n_hosts)
    hosts = L.host_addrs((seed % 97) * 10_000_000, n_hosts)
    salts = L.peer_salts(seed, n_hosts)
    own = bases is None
    if own:
        bases = make_backgrounds(params, seed)
    n_backgrounds = len(bases)
    # streams: consecutive hosts up to hosts_per_stream and the peer budget
    chunks, a = [], 0
    while a < n_hosts:
        b, tot = a, 0
        while b < n_hosts and b - a < hosts_per_stream and (b == a or tot + cards[b] <= peer_budget):
            tot += int(cards[b])
            b += 1
        chunks.append((a, b))
        a = b
    gen = L.PlantedGenerator(max(peer_budget, int(cards.max())) + 1, law=law)
    work = sps.Sketch(params)
    feats = torch.zeros((n_hosts, WINDOW), dtype=torch.int32, device="cuda")
    res = torch.zeros(n_hosts * 24, dtype=torch.uint8, device="cuda")
    hosts_d = torch.from_numpy(hosts.view(np.int32)).cuda()
    for k, (a, b) in enumerate(chunks):
        work.reset()
        buckets = gen.generate(hosts[a:b], cards[a:b], salts[a:b], key=seed * 1_000_003 + k)
        for s in range(1, WINDOW + 1):
            sps.sps_ingest(work.h, buckets[s - 1], s)
        work.merge([bases[k % n_backgrounds]])
        hd = hosts_d[a:b]
        sps.sps_features(work.h, hd, WINDOW, feats[a:b])
        r = sps.sps_estimate_hosts(work.h, hd, WINDOW)
        res[a * 24:b * 24].copy_(r[: (b - a) * 24])
        if log and (k % 500 == 0 or k == len(chunks) - 1):
            log(f"dataset {seed:#x}: stream {k + 1}/{len(chunks)}")
    torch.cuda.synchronize()
    r = sps.results_to_numpy(res, n_hosts)
    if own:
        for s in bases:
            s.close()
    work.close()
    return Dataset(feats.cpu().numpy().view(np.uint32), cards, r["estimate"].copy(),
                   r["flags"].copy(), params["etap"])


def init_weights(seed: int) -> np.ndarray:
    """He-normal weights, zero biases, flattened in the library's parameter order."""
    g = np.random.Generator(np.random.Philox(seed))
    parts = []
    for shape, fan_in, is_w in [((64, 10), 10, True), ((64,), 0, False), ((64, 64), 64, True),
                                ((64,), 0, False), ((1, 64), 64, True), ((1,), 0, False)]:
        parts.append((g.standard_normal(shape) * math.sqrt(2.0 / fan_in)).ravel() if is_w
                     else np.zeros(int(np.prod(shape))))
    w = np.concatenate(parts).astype(np.float32)
    assert w.size == sps.MLP_PARAMS
    return w


def informative(ds: Dataset) -> np.ndarray:
    """Hosts whose newest age is not saturated: the only ones the network may estimate."""
    return ds.features[:, 0] < ds.etap - 1


def train(ds: Dataset, epochs: int = 30, batch: int = 4096, lr: float = 3e-3, seed: int = 1,
          log=None) -> torch.Tensor:
    """Adam on the mean squared error of log-cardinality over the informative hosts; returns
    device float32 weights."""
    keep = informative(ds)
    feats = np.ascontiguousarray(ds.features[keep])
    n = feats.shape[0]
    feat = torch.from_numpy(feats.view(np.int32)).cuda()
    target = torch.from_numpy(np.log(ds.cards[keep].astype(np.float64)).astype(np.float32)).cuda()
    w = torch.from_numpy(init_weights(seed)).cuda()
    m = torch.zeros_like(w)
    v = torch.zeros_like(w)
    grad = torch.zeros_like(w)
    loss = torch.zeros(1, dtype=torch.float32, device="cuda")
    work = torch.empty(sps.sps_mlp_work_bytes(batch), dtype=torch.uint8, device="cuda")
    g = np.random.Generator(np.random.Philox(seed ^ 0xE90C))
    step = 0
    steps_per_epoch = max(1, n // batch)
    total = epochs * steps_per_epoch
    for ep in range(epochs):
        perm = torch.from_numpy(g.permutation(n).astype(np.int32)).cuda()
        acc = torch.zeros(1, dtype=torch.float32, device="cuda")
        for i in range(steps_per_epoch):
            idx = perm[i * batch:(i + 1) * batch]
            nb = idx.numel()
            sps.sps_mlp_grad(w, feat, target, idx, nb, ds.etap, work, grad, loss)
            step += 1
            # cosine decay to 5% of the base rate
            lr_t = lr * (0.05 + 0.95 * 0.5 * (1 + math.cos(math.pi * step / total)))
            sps.sps_mlp_adam(w, m, v, grad, step, lr_t)
            acc += loss
        if log and (ep % 5 == 0 or ep == epochs - 1):
            log(f"epoch {ep + 1}/{epochs}: mse(log) = {float(acc.item()) / steps_per_epoch:.4f}")
    return w


def predict(w: torch.Tensor, ds: Dataset, bf16: bool = True) -> np.ndarray:
    n = ds.features.shape[0]
    feat = torch.from_numpy(np.ascontiguousarray(ds.features).view(np.int32)).cuda()
    y = torch.zeros(n, dtype=torch.float32, device="cuda")
    sps.sps_mlp_forward(w, feat, n, ds.etap, bf16, y)
    return y.cpu().numpy().astype(np.float64)


@dataclasses.dataclass
class Gate:
    lo: np.ndarray        # per-feature training minimum (of x / eta')
    hi: np.ndarray        # per-feature training maximum
    min_live: int         # the network is used only when |USLE|^k >= min_live
    max_card: float


def gated(ds: Dataset, y: np.ndarray, gate: Gate) -> tuple:
    """Estimates the scan would report with the network attached (mirrors the kernel's rule)."""
    f = ds.features.astype(np.float32) / np.float32(ds.etap)
    in_range = np.all((f >= gate.lo) & (f <= gate.hi), axis=1)
    use = (ds.features[:, -1] >= gate.min_live) & in_range & informative(ds) & \
        (y >= 0) & (y <= math.log(gate.max_card))
    net = np.exp(y.astype(np.float32)).astype(np.float64)
    # a saturated linear count is the largest value it can express: the network only raises it
    sat = (ds.lc_flags & sps.F_SATURATED) != 0
    net = np.where(sat & (net < ds.lc), ds.lc, net)
    return np.where(use, net, ds.lc), use


def fit_gate(train_ds: Dataset, val: Dataset, y_val: np.ndarray, max_card: float = 1e6) -> Gate:
    """Feature ranges from the training set; min_live chosen on the validation set to minimise
    the mean relative error."""
    f = train_ds.features[informative(train_ds)].astype(np.float32) / np.float32(train_ds.etap)
    lo, hi = f.min(0), f.max(0)
    best = None
    for ml in [0, 64, 128, 256, 384, 512, 640, 768, 832, 896, 960, 992, 1008, 1016, 1020, 1023,
               10 ** 9]:
        gate = Gate(lo, hi, ml, max_card)
        est, _ = gated(val, y_val, gate)
        err = float(np.mean(np.abs(est - val.cards) / val.cards))
        if best is None or err < best[0]:
            best = (err, gate)
    return best[1]


def rel_err_table(cards: np.ndarray, est: np.ndarray) -> list:
    rows = []
    for lo, hi in DECADES:
        sel = (cards >= lo) & (cards < hi)
        rows.append({"decade": f"[{lo},{hi})", "n": int(sel.sum()),
                     "mean_rel_err": float(np.mean(np.abs(est[sel] - cards[sel]) / cards[sel]))
                     if sel.any() else None})
    return rows


def attach(sketch_handle, w: torch.Tensor, gate: Gate):
    sps.sps_attach_mlp(sketch_handle, w, gate.lo, gate.hi, gate.min_live, gate.max_card)
