"""Seeded synthetic packet streams for the sliding super point workloads.

This module holds no arithmetic of the method (no sketch hashes, no estimators): it only
draws (src, dst) address pairs with the shapes and distributions of the workloads, so the
CPU oracle and the GPU path can be fed the same bytes.  The paper evaluates on a CAIDA OC192
trace (Sec. 5) that is not available here; these streams stand in for it.

Recipe (common to every workload):
  * RNG: numpy's Philox4x32-10 bit generator (Salmon et al., SC'11), seeded per workload.
  * Host addresses: rank rho in [1, N] -> addr_mix(rho, HOST_SALT), a bijection on 32 bits,
    so addresses spread over all 32 bits.  Planted hosts use ranks above N (disjoint).
  * Background peers: u uniform in [0, 2^24) -> addr_mix(u, PEER_SALT).
  * Planted peers of planted host j: addr_mix(((j + 1) << 24) | t, PEER_SALT) for a per-host
    counter t, so every planted packet carries a fresh peer, disjoint from the background.
  * Zipf: exact inverse-CDF sampling over N ranks with exponent s.
  * Slices: equal packet counts, the remainder going to the first slices; each slice holds
    ceil(c_j / k) packets of every planted host j; the background fills the rest; packets
    are shuffled within each slice.

Packets are an (n, 2) uint32 array: column 0 = src, column 1 = dst (the 8-byte pair layout).
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np
import torch

HOST_SALT = np.uint32(0x5EED0001)
PEER_SALT = np.uint32(0x5EED0002)


def addr_mix(x, salt) -> np.ndarray:
    """Bijective 32-bit scramble used only to spread synthetic addresses (not a sketch hash).

    xor salt; odd multiply; xorshift; odd multiply; xorshift -- every step is invertible
    modulo 2^32, so distinct inputs give distinct addresses."""
    v = np.asarray(x, dtype=np.uint32) ^ np.uint32(salt)
    with np.errstate(over="ignore"):
        v = v * np.uint32(0x2C1B3C6D)
        v ^= v >> np.uint32(12)
        v = v * np.uint32(0x297A2D39)
        v ^= v >> np.uint32(15)
    return v.astype(np.uint32)


def zipf_cdf(n_ranks: int, s: float) -> torch.Tensor:
    """Cumulative probabilities of ranks 1..n_ranks with weight rank^-s (float64)."""
    w = torch.arange(1, n_ranks + 1, dtype=torch.float64).pow(-s)
    c = torch.cumsum(w, 0)
    return c / c[-1]


def zipf_ranks(rng: np.random.Generator, cdf: torch.Tensor, n: int) -> np.ndarray:
    """n Zipf ranks in [1, len(cdf)] by inverse-CDF lookup."""
    u = torch.from_numpy(rng.random(n))
    idx = torch.searchsorted(cdf, u, right=True).clamp_(max=cdf.numel() - 1)
    return idx.numpy().astype(np.uint32) + np.uint32(1)


@dataclasses.dataclass
class StreamRecipe:
    name: str
    seed: int
    n_packets: int
    n_slices: int
    window: int
    n_hosts: int
    zipf_s: float
    planted: list  # target distinct peers per full window, one entry per planted host


@dataclasses.dataclass
class Stream:
    recipe: StreamRecipe
    pkts: np.ndarray          # (n, 2) uint32, slice-major
    slice_off: np.ndarray     # (n_slices + 1,) int64 offsets into pkts
    planted_hosts: np.ndarray  # (n_planted,) uint32 addresses
    planted_per_slice: np.ndarray  # (n_planted,) packets per slice of each planted host

    def slice_pkts(self, s: int) -> np.ndarray:
        """Packets of slice s (slices are numbered from 1)."""
        return self.pkts[self.slice_off[s - 1]:self.slice_off[s]]


def slice_sizes(n_packets: int, n_slices: int) -> np.ndarray:
    base = n_packets // n_slices
    sizes = np.full(n_slices, base, dtype=np.int64)
    sizes[: n_packets - base * n_slices] += 1
    return sizes


def make_stream(rec: StreamRecipe) -> Stream:
    """Generate a whole stream, slice by slice."""
    rng = np.random.Generator(np.random.Philox(rec.seed))
    cdf = zipf_cdf(rec.n_hosts, rec.zipf_s)
    planted = np.asarray(rec.planted, dtype=np.int64)
    n_pl = len(planted)
    per_slice = np.ceil(planted / rec.window).astype(np.int64) if n_pl else np.zeros(0, np.int64)
    planted_hosts = addr_mix(np.arange(rec.n_hosts + 1, rec.n_hosts + 1 + n_pl, dtype=np.uint64)
                             .astype(np.uint32), HOST_SALT)
    sizes = slice_sizes(rec.n_packets, rec.n_slices)
    pl_total = int(per_slice.sum())
    if (sizes < pl_total).any():
        raise ValueError("planted packets exceed a slice")
    pkts = np.empty((rec.n_packets, 2), dtype=np.uint32)
    off = np.zeros(rec.n_slices + 1, dtype=np.int64)
    off[1:] = np.cumsum(sizes)
    # planted: host j emits per_slice[j] packets per slice with fresh peers (counter t)
    pl_dst = np.repeat(planted_hosts, per_slice)
    pl_j = np.repeat(np.arange(n_pl, dtype=np.uint32), per_slice)
    pl_t_base = np.concatenate([np.arange(m, dtype=np.uint32) for m in per_slice]) if n_pl else \
        np.zeros(0, np.uint32)
    for s in range(rec.n_slices):
        nb = int(sizes[s]) - pl_total
        bg_dst = addr_mix(zipf_ranks(rng, cdf, nb), HOST_SALT)
        bg_src = addr_mix(rng.integers(0, 1 << 24, size=nb, dtype=np.uint32), PEER_SALT)
        t = pl_t_base + (np.repeat(per_slice, per_slice).astype(np.uint32) * np.uint32(s)
                         if n_pl else np.zeros(0, np.uint32))
        pl_src = addr_mix(((pl_j + np.uint32(1)) << np.uint32(24)) | t, PEER_SALT)
        src = np.concatenate([bg_src, pl_src])
        dst = np.concatenate([bg_dst, pl_dst])
        perm = rng.permutation(src.shape[0])
        blk = pkts[off[s]:off[s + 1]]
        blk[:, 0] = src[perm]
        blk[:, 1] = dst[perm]
    return Stream(rec, pkts, off, planted_hosts, per_slice)


def log_uniform_int(rng: np.random.Generator, lo: float, hi: float, n: int) -> list:
    return [int(round(math.exp(v))) for v in rng.uniform(math.log(lo), math.log(hi), n)]


@dataclasses.dataclass
class MultiRecipe:
    """m routers that see one host population.  Router j's background packet count over the
    whole run is T_j = round(median * exp(sigma * Z_j)), Z_j ~ N(0, 1); every planted host
    emits ceil(c / window) fresh peers per slice, each packet to a uniformly drawn router
    (so only the merged view holds a planted host's full cardinality).  Planted packets come
    on top of the background counts."""
    name: str
    seed: int
    n_routers: int
    median: int
    sigma: float
    n_slices: int
    window: int
    n_hosts: int
    zipf_s: float
    planted: list


def router_totals(rec: MultiRecipe) -> np.ndarray:
    rng = np.random.Generator(np.random.Philox(rec.seed ^ 0x7070))
    z = rng.standard_normal(rec.n_routers)
    return np.round(rec.median * np.exp(rec.sigma * z)).astype(np.int64)


def make_multi_stream(rec: MultiRecipe) -> list:
    """One Stream per router (slices numbered from 1)."""
    rng = np.random.Generator(np.random.Philox(rec.seed))
    cdf = zipf_cdf(rec.n_hosts, rec.zipf_s)
    totals = router_totals(rec)
    planted = np.asarray(rec.planted, dtype=np.int64)
    n_pl = len(planted)
    per_slice = np.ceil(planted / rec.window).astype(np.int64) if n_pl else np.zeros(0, np.int64)
    planted_hosts = addr_mix(np.arange(rec.n_hosts + 1, rec.n_hosts + 1 + n_pl, dtype=np.uint64)
                             .astype(np.uint32), HOST_SALT)
    pl_dst = np.repeat(planted_hosts, per_slice)
    pl_j = np.repeat(np.arange(n_pl, dtype=np.uint32), per_slice)
    pl_t_base = (np.concatenate([np.arange(m, dtype=np.uint32) for m in per_slice]) if n_pl
                 else np.zeros(0, np.uint32))
    bg_sizes = [slice_sizes(int(t), rec.n_slices) for t in totals]
    chunks = [[] for _ in range(rec.n_routers)]
    for s in range(rec.n_slices):
        t = pl_t_base + (np.repeat(per_slice, per_slice).astype(np.uint32) * np.uint32(s)
                         if n_pl else np.zeros(0, np.uint32))
        pl_src = addr_mix(((pl_j + np.uint32(1)) << np.uint32(24)) | t, PEER_SALT)
        who = rng.integers(0, rec.n_routers, size=pl_src.shape[0])
        for r in range(rec.n_routers):
            nb = int(bg_sizes[r][s])
            bg_dst = addr_mix(zipf_ranks(rng, cdf, nb), HOST_SALT)
            bg_src = addr_mix(rng.integers(0, 1 << 24, size=nb, dtype=np.uint32), PEER_SALT)
            mine = who == r
            src = np.concatenate([bg_src, pl_src[mine]])
            dst = np.concatenate([bg_dst, pl_dst[mine]])
            perm = rng.permutation(src.shape[0])
            chunks[r].append(np.stack([src[perm], dst[perm]], 1))
    out = []
    for r in range(rec.n_routers):
        sizes = np.array([c.shape[0] for c in chunks[r]], dtype=np.int64)
        off = np.zeros(rec.n_slices + 1, dtype=np.int64)
        off[1:] = np.cumsum(sizes)
        srec = StreamRecipe(f"{rec.name}/router{r}", rec.seed, int(off[-1]), rec.n_slices,
                            rec.window, rec.n_hosts, rec.zipf_s, list(rec.planted))
        out.append(Stream(srec, np.concatenate(chunks[r]), off, planted_hosts, per_slice))
    return out
