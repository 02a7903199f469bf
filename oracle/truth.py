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
