"""Workload definitions: stream recipes plus the sketch parameters each workload runs with.

Sketch parameter names follow the paper: SRE array of 2^q columns x r rows with eta cells per
SRE and RHFG shift step delta; SLE array of 2^q' SLEs x r' rows with eta' cells per SLE and
offset delta' between adjacent SLEs; theta fixes the sampling depth tau (Eq. 1).
Values the workload statement leaves open are chosen in the design notes (rows, shift step,
cell sharing); (r - 2) * delta + q = 32 in every workload (the RHFG coverage condition).
"""
from __future__ import annotations

import numpy as np

from . import MultiRecipe, StreamRecipe, log_uniform_int


def sketch_params(q, r, delta, eta, qp, rp, etap, deltap, theta, seed, anet_side=0):
    return dict(q=q, r=r, delta=delta, eta=eta, qp=qp, rp=rp, etap=etap, deltap=deltap,
                theta=theta, anet_side=anet_side, seed=seed)


# Plain method, one router: 2^20 packets over 10 slices, window 5, threshold 1024.
C1_RECIPE = StreamRecipe(name="c1_plain_1router", seed=0x180509246001, n_packets=1 << 20,
                         n_slices=10, window=5, n_hosts=1 << 16, zipf_s=1.1,
                         planted=[2000, 3175, 5040, 8000])
C1_PARAMS = sketch_params(q=12, r=6, delta=5, eta=8, qp=12, rp=5, etap=1024, deltap=1024,
                          theta=1024, seed=0x5A5A180509246001)
C1_WINDOW, C1_THRESHOLD = 5, 1024.0


def _c2_planted():
    rng = np.random.Generator(np.random.Philox(0x180509246002 ^ 0xFACE))
    return log_uniform_int(rng, 1e3, 1e5, 200)


# Single router at scale: 2^26 packets over 60 slices, window 10, threshold 1024.
C2_RECIPE = StreamRecipe(name="c2_single_router_scale", seed=0x180509246002,
                         n_packets=1 << 26, n_slices=60, window=10, n_hosts=1 << 22,
                         zipf_s=1.05, planted=_c2_planted())
C2_PARAMS = sketch_params(q=14, r=11, delta=2, eta=8, qp=16, rp=5, etap=1024, deltap=1024,
                          theta=1024, seed=0x5A5A180509246002)
C2_WINDOW, C2_THRESHOLD = 10, 1024.0

# Same sketch shapes on a short stream: the parity tests' small case of the scale workload.
C2_SMALL_RECIPE = StreamRecipe(name="c2_shape_small_stream", seed=0x180509246012,
                               n_packets=3 << 20, n_slices=12, window=10, n_hosts=1 << 22,
                               zipf_s=1.05, planted=[1500, 3000, 6000, 12000, 40000])


def _c3_planted():
    rng = np.random.Generator(np.random.Philox(0x180509246003 ^ 0xFACE))
    return log_uniform_int(rng, 1e3, 1e5, 200)


# Distributed merge on one GPU: 16 routers, lognormal packet counts (median 2^22, sigma 1)
# over 30 slices; merged by element-wise max, scanned with window 10 and threshold 2048.
C3_RECIPE = MultiRecipe(name="c3_distributed_merge_16", seed=0x180509246003, n_routers=16,
                        median=1 << 22, sigma=1.0, n_slices=30, window=10, n_hosts=1 << 22,
                        zipf_s=1.05, planted=_c3_planted())
C3_PARAMS = sketch_params(q=17, r=10, delta=2, eta=8, qp=16, rp=5, etap=1024, deltap=1024,
                          theta=2048, seed=0x5A5A180509246003)
C3_WINDOW, C3_THRESHOLD = 10, 2048.0

# The same sketch shapes with small routers: the parity tests' case of the merge workload.
C3_SMALL_RECIPE = MultiRecipe(name="c3_shape_small", seed=0x180509246013, n_routers=16,
                              median=1 << 17, sigma=1.0, n_slices=12, window=10,
                              n_hosts=1 << 20, zipf_s=1.05, planted=[3000, 8000, 20000, 60000])

# Serving loop: 64 routers, Poisson batch arrivals at 2e9 packets/s (batches 4 Ki..4 Mi),
# 120 slices of 10 ms, window 10, threshold 1024; all sketches resident (12 GiB budget).
C4_PARAMS = sketch_params(q=14, r=11, delta=2, eta=8, qp=14, rp=5, etap=1024, deltap=1024,
                          theta=1024, seed=0x5A5A180509246004)
C4_WINDOW, C4_THRESHOLD = 10, 1024.0
C4_ROUTERS, C4_RATE, C4_SLICE_S, C4_SLICES, C4_BUDGET = 64, 2e9, 0.010, 120, 12 << 30
C4_SEED = 0x180509246004

# Learned estimator: 1e6 training hosts, window 10, SLE array 5 x 65536 x 1024.
C5_PARAMS = sketch_params(q=14, r=11, delta=2, eta=8, qp=16, rp=5, etap=1024, deltap=1024,
                          theta=1024, seed=0x5A5A180509246005)
C5_TRAIN, C5_VAL, C5_TEST = 1_000_000, 50_000, 100_000
C5_SEEDS = (0x180509246005, 0x180509246015, 0x180509246025)
