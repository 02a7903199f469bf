"""Learned-estimator workload: hosts with known cardinalities embedded in background traffic.

Recipe (stands in for labelled traffic, which the paper does not have either):
  * cardinalities c = max(1, round(exp(U[0, ln c_max]))), log-uniform over 1..c_max;
  * every host's peers are distinct; a peer first appears in a slice drawn uniformly from the
    window and appears again in every later slice with probability 0.3 (arrival law 0, the
    training law); law 1 -- the scale workload's planted hosts, for evaluation away from the
    training law -- spreads fresh peers evenly over the slices, peer i only in slice
    1 + (i mod window);
  * hosts are embedded a few hundred per stream into background streams of the scale
    workload's density (Zipf 1.05 over 2^22 hosts, 1,118,481 packets per slice);
  * a max-of-stamps sketch only keeps a peer's last appearance, so each peer contributes one
    packet, stamped with its last slice.

The GPU generator (csrc/synth_gen.hip -> libsynth.so) and the numpy twin here draw the same
packets from the same counter-based generator (SplitMix64 outputs addressed by counter).
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

from . import HOST_SALT, PEER_SALT, StreamRecipe, addr_mix

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libsynth.so")
GAMMA = np.uint64(0x9E3779B97F4A7C15)
REPEAT = 1288490189  # round(0.3 * 2^32)
WINDOW = 10
BACKGROUND_PER_SLICE = 1118481
HOST_RANK_BASE = (1 << 22) + 1 + 1000  # above the background ranks and the other workloads


def _mix64(z: np.ndarray) -> np.ndarray:
    with np.errstate(over="ignore"):
        z = (z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
        z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
        return z ^ (z >> np.uint64(31))


def rng(key: int, ctr: np.ndarray) -> np.ndarray:
    """SplitMix64 output number ctr+1 from seed `key` (vectorised)."""
    ctr = np.asarray(ctr, dtype=np.uint64)
    with np.errstate(over="ignore"):
        return _mix64(np.uint64(key) + (ctr + np.uint64(1)) * GAMMA)


def draw_cards(seed: int, n: int, c_max: float = 1e6) -> np.ndarray:
    g = np.random.Generator(np.random.Philox(seed))
    return np.maximum(1, np.round(np.exp(g.uniform(0.0, np.log(c_max), n)))).astype(np.int64)


def host_addrs(first_index: int, n: int) -> np.ndarray:
    ranks = np.arange(HOST_RANK_BASE + first_index, HOST_RANK_BASE + first_index + n,
                      dtype=np.uint64).astype(np.uint32)
    return addr_mix(ranks, HOST_SALT)


def peer_salts(key: int, n: int) -> np.ndarray:
    return (rng(key ^ 0x5A17, np.arange(n)) >> np.uint64(32)).astype(np.uint32)


def background_recipe(seed: int) -> StreamRecipe:
    return StreamRecipe(name=f"learn_background_{seed:x}", seed=seed,
                        n_packets=WINDOW * BACKGROUND_PER_SLICE, n_slices=WINDOW, window=WINDOW,
                        n_hosts=1 << 22, zipf_s=1.05, planted=[])


def planted_cpu(hosts, cards, salts, key: int, window: int = WINDOW, law: int = 0):
    """Numpy twin of the GPU generator: per-slice (n, 2) packet arrays, rows sorted."""
    cards = np.asarray(cards, dtype=np.int64)
    prefix = np.zeros(len(cards) + 1, dtype=np.int64)
    prefix[1:] = np.cumsum(cards)
    g = np.arange(prefix[-1], dtype=np.uint64)
    j = np.repeat(np.arange(len(cards)), cards)
    i = (g - prefix[j].astype(np.uint64)).astype(np.uint32)
    with np.errstate(over="ignore"):
        src = addr_mix((i + salts[j]).astype(np.uint32), PEER_SALT)
    dst = np.asarray(hosts, dtype=np.uint32)[j]
    if law == 1:
        last = 1 + (i.astype(np.int64) % window)
    else:
        u = (rng(key, g * np.uint64(16)) >> np.uint64(32)).astype(np.uint64)
        f = (np.uint64(1) + ((u * np.uint64(window)) >> np.uint64(32))).astype(np.int64)
        last = f.copy()
        for s in range(2, window + 1):
            hit = (rng(key, g * np.uint64(16) + np.uint64(s)) >> np.uint64(32)) < \
                np.uint64(REPEAT)
            last = np.where((s > f) & hit, s, last)
    out = []
    for s in range(1, window + 1):
        sel = last == s
        p = np.stack([src[sel], dst[sel]], 1)
        out.append(p[np.lexsort((p[:, 0], p[:, 1]))] if len(p) else p)
    return out


# ---------------------------------------------------------------- GPU generator
def build(verbose: bool = False) -> str:
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    cmd = [hipcc, "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
           "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
           os.path.join(HERE, "csrc", "synth_gen.hip"), "-o", LIB_PATH + ".tmp"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(LIB_PATH + ".tmp", LIB_PATH)
    return LIB_PATH


_lib = None


def _glib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} missing: run __graft_entry__.build()")
        L = C.CDLL(LIB_PATH)
        vp = C.c_void_p
        L.synth_gen_planted.argtypes = [vp, vp, vp, C.c_uint32, C.c_uint64, C.c_uint32,
                                        C.c_uint32, C.c_uint32, vp, C.c_uint64, vp, vp]
        L.synth_gen_planted.restype = C.c_int
        _lib = L
    return _lib


class PlantedGenerator:
    """Generates one stream's planted packets on the GPU into per-slice buckets."""

    def __init__(self, max_peers: int, window: int = WINDOW, device="cuda", law: int = 0):
        import torch
        self.window = window
        self.law = law
        self.cap = int(max_peers)
        self.buf = torch.empty((window, self.cap, 2), dtype=torch.int32, device=device)
        self.counts = torch.zeros(window, dtype=torch.int64, device=device)

    def generate(self, hosts, cards, salts, key: int, stream=None):
        """hosts, salts: uint32 numpy arrays; cards: int64.  Returns a list of per-slice
        device tensors (views into the bucket buffer)."""
        import torch
        cards = np.asarray(cards, dtype=np.int64)
        total = int(cards.sum())
        if total > self.cap:
            raise ValueError("stream exceeds the generator capacity")
        prefix = np.zeros(len(cards) + 1, dtype=np.uint64)
        prefix[1:] = np.cumsum(cards)
        dev = self.buf.device
        h = torch.from_numpy(np.ascontiguousarray(hosts, dtype=np.uint32).view(np.int32)).to(dev)
        pf = torch.from_numpy(prefix.view(np.int64)).to(dev)
        sl = torch.from_numpy(np.ascontiguousarray(salts, dtype=np.uint32).view(np.int32)).to(dev)
        self.counts.zero_()
        st = stream if stream is not None else torch.cuda.current_stream()
        rc = _glib().synth_gen_planted(
            C.c_void_p(h.data_ptr()), C.c_void_p(pf.data_ptr()), C.c_void_p(sl.data_ptr()),
            len(cards), key, self.window, int(PEER_SALT), self.law, C.c_void_p(self.buf.data_ptr()),
            self.cap, C.c_void_p(self.counts.data_ptr()), C.c_void_p(st.cuda_stream))
        if rc:
            raise RuntimeError(f"synth_gen_planted: {rc}")
        n = self.counts.cpu().numpy()
        return [self.buf[s, : int(n[s])] for s in range(self.window)]
