"""Exact sliding-window cardinalities -- TEST INFRASTRUCTURE ONLY (part of the oracle).

Def. 1-2 of the paper: the opposite-host set OH(aip, t, k) holds every bip that shares a
packet with aip in the k slices of the window; aip is a sliding super point when
|OH| >= theta.  Computed here exactly with sorted unique pair keys, no sketch involved.
"""
from __future__ import annotations

import numpy as np


def window_pairs(stream, cur: int, k: int, anet_side: int = 0) -> np.ndarray:
    """Packets of the window of k slices ending at slice `cur` (slices numbered from 1)."""
    lo = max(1, cur - k + 1)
    return stream.pkts[stream.slice_off[lo - 1]:stream.slice_off[cur]]


def cardinalities(pkts: np.ndarray, anet_side: int = 0):
    """(hosts ascending, distinct opposite-host counts) over a packet set."""
    src = pkts[:, 0].astype(np.uint64)
    dst = pkts[:, 1].astype(np.uint64)
    aip, bip = (dst, src) if anet_side == 0 else (src, dst)
    keys = np.unique((aip << np.uint64(32)) | bip)
    hosts, counts = np.unique((keys >> np.uint64(32)).astype(np.uint32), return_counts=True)
    return hosts, counts


def super_points(stream, cur: int, k: int, theta: float, anet_side: int = 0):
    hosts, counts = cardinalities(window_pairs(stream, cur, k), anet_side)
    keep = counts >= theta
    return hosts[keep], counts[keep]


def detection_rates(true_hosts, reported_hosts):
    """Def. 5: FPR = N+/N, FNR = N-/N, TFR = FPR + FNR (N = number of true super points)."""
    t = set(int(h) for h in true_hosts)
    r = set(int(h) for h in reported_hosts)
    n = max(1, len(t))
    fpr = len(r - t) / n
    fnr = len(t - r) / n
    return fpr, fnr, fpr + fnr


def sliding_cardinalities(stream, windows, theta_min: float, anet_side: int = 0):
    """|OH(aip)| over every window of the stream at once (Def. 1-2, W(t, k)), for the hosts
    that can reach theta_min in some window.

    Returns {k: (hosts, counts)} with counts[h, cur - 1] = number of distinct opposite hosts
    of hosts[h] in the window of k slices ending at slice cur (cur = 1 .. n_slices; windows
    that start before slice 1 hold the slices from 1).  A host whose distinct opposite hosts
    over the whole stream number fewer than theta_min is left out (no window can exceed
    that).  Method: each distinct (aip, bip) pair with its distinct slices s_1 < s_2 < ...;
    the window ending at cur holds the pair iff some s_j lies in [cur - k + 1, cur], so
    occurrence s_j newly covers the window ends [max(s_j, s_{j-1} + k), s_j + k - 1] --
    ranges that partition the covered ends, summed per host with a difference array."""
    n_sl = len(stream.slice_off) - 1
    keys, sl = [], []
    for s in range(1, n_sl + 1):
        p = stream.slice_pkts(s)
        src = p[:, 0].astype(np.uint64)
        dst = p[:, 1].astype(np.uint64)
        aip, bip = (dst, src) if anet_side == 0 else (src, dst)
        u = np.unique((aip << np.uint64(32)) | bip)
        keys.append(u)
        sl.append(np.full(u.shape[0], s, dtype=np.int32))
    keys = np.concatenate(keys)
    sl = np.concatenate(sl)
    order = np.argsort(keys, kind="stable")  # slices stay ascending within a pair
    keys = keys[order]
    sl = sl[order]
    del order
    host = (keys >> np.uint64(32)).astype(np.uint32)
    first = np.ones(keys.shape[0], dtype=bool)
    first[1:] = keys[1:] != keys[:-1]
    del keys
    # distinct opposite hosts of each host over the whole stream
    uh, total = np.unique(host[first], return_counts=True)
    hosts = uh[total >= theta_min]
    if len(hosts):
        pos = np.minimum(np.searchsorted(hosts, host), len(hosts) - 1)
        sel = hosts[pos] == host
    else:
        pos = np.zeros(host.shape, dtype=np.int64)
        sel = np.zeros(host.shape, dtype=bool)
    prev = np.empty_like(sl)
    prev[0] = 0
    prev[1:] = sl[:-1]
    out = {}
    for k in windows:
        a = np.where(first, sl, np.maximum(sl, prev + k))
        b = np.minimum(sl + k - 1, n_sl)
        m = sel & (a <= b)
        diff = np.zeros((len(hosts), n_sl + 2), dtype=np.int64)
        np.add.at(diff, (pos[m], a[m]), 1)
        np.add.at(diff, (pos[m], b[m] + 1), -1)
        out[k] = (hosts, np.cumsum(diff, axis=1)[:, 1:n_sl + 1])
    return out


def sliding_super_points(card, k: int, cur: int, theta: float):
    """Hosts (ascending) and counts with |OH| >= theta in the window of k slices ending at cur,
    from the output of sliding_cardinalities."""
    hosts, counts = card[k]
    c = counts[:, cur - 1]
    keep = c >= theta
    return hosts[keep], c[keep]
