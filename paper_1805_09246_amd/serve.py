"""Serving loop: many routers' sketches resident on one GPU, fed by continuous batching.

Routers submit packet batches at any time.  Every slice (a fixed wall-clock period) the loop
takes everything that has arrived so far -- whatever arrived while the previous slice was
on the GPU joins this one -- and launches one captured graph: a single batched ingest of all
those batches into their routers' sketches (sps_ingest_batched), then a scan of every
resident router (sps_scan_async).  The graph of slice s runs while batches for slice s+1
accumulate.  Behind each slice's graph the stream runs a host notification
(sps_stream_host_time) that stores the host clock when the slice's GPU work has finished;
results are copied back and filed as reports by `collect`, which the loop calls between
launches.  Latency of a batch is the time from its arrival to the completion of the slice
that ingested it (`latencies`, independent of when the loop gets round to collecting);
`report_latencies` run to the filing of the report.  Times are CLOCK_MONOTONIC seconds.

Each of the `depth` result buffers has its own executable graph.  A new slice's capture is
applied to the buffer's graph in place when only kernel arguments changed (the usual case:
the same number of batched-ingest launches and resident routers); otherwise that graph is
instantiated again.  Host time of capture, update and instantiation is recorded per slice.

Routers are admitted while their sketch fits the device-memory budget; a router that cannot
be admitted waits (its batches are held) until a resident router leaves and frees a slot.
Slots are reused: a freed sketch is reset and handed to the next router.

Stamps are u16 slice numbers, so before the internal slice number would pass 65534 every
resident sketch is rebased (sps_rebase) by the same offset, keeping the newest `window`
slices; reports keep counting slices from the start of serving.
"""
from __future__ import annotations

import collections
import dataclasses
import threading
import time

import numpy as np
import torch

from . import sps


def now() -> float:
    """Host clock of arrivals and completions: CLOCK_MONOTONIC seconds (the clock the
    library's stream notification reads)."""
    return time.clock_gettime(time.CLOCK_MONOTONIC)


@dataclasses.dataclass
class Report:
    router: int
    slice: int
    results: np.ndarray        # sps_result records, ascending by host
    batches: int
    packets: int
    latencies: list            # seconds, one per batch ingested in this slice: arrival to the
                               # completion of the slice's work on the GPU
    info_flags: int = 0        # scan info flags: bit 0 candidate list overflowed its capacity,
                               # bit 1 more hosts kept than the result buffer holds
    kept: int = 0              # hosts the scan kept (results holds min(kept, result_cap))
    report_latencies: list = dataclasses.field(default_factory=list)  # arrival to report

    @property
    def complete(self) -> bool:
        """False when the scan overflowed a buffer and `results` is truncated."""
        return self.info_flags == 0


class Slot:
    def __init__(self, params: dict, index: int):
        self.sketch = sps.Sketch(params)
        self.index = index
        self.router = None


class Server:
    """depth: slices allowed on the GPU at once (results are double-buffered by slice)."""

    def __init__(self, params: dict, window: int, threshold: float, budget_bytes: int,
                 result_cap: int = 4096, use_graph: bool = True, depth: int = 2,
                 start_slice: int = 0):
        self.params = dict(params)
        self.window = window
        self.threshold = threshold
        self.budget = int(budget_bytes)
        self.cap = result_cap
        self.use_graph = use_graph
        self.depth = depth
        self.sketch_bytes = sps.sps_sketch_bytes(params)
        self.max_slots = max(0, self.budget // self.sketch_bytes)
        nb = max(1, self.max_slots)
        # per-slice result buffers, all slots side by side: one copy back per slice
        self.res = torch.zeros((depth, nb, result_cap * 24), dtype=torch.uint8, device="cuda")
        self.info = torch.zeros((depth, nb, 8), dtype=torch.int32, device="cuda")
        self.slots: list[Slot] = []
        self.free: list[Slot] = []
        self.by_router: dict[int, Slot] = {}
        self.waiting = collections.deque()        # routers not yet admitted
        self.held = collections.defaultdict(list)  # batches of waiting routers
        self.pending = []                           # (slot, pkts, arrival time)
        self.lock = threading.Lock()
        self.stream = torch.cuda.Stream()
        self.slice_no = start_slice   # internal slice number (the sketches' time base)
        self.slice_base = 0            # slices shifted out by rebases
        self.rebases = 0
        self.reports: list[Report] = []
        self.refused = 0
        self.incomplete = 0        # reports whose scan overflowed a buffer
        self.graphs = [None] * depth          # one executable graph per result buffer
        self.host_ms = {"capture": [], "update": [], "instantiate": []}
        self.inflight = collections.deque()

    # ---------------------------------------------------------------- admission
    def used_bytes(self) -> int:
        return len(self.slots) * self.sketch_bytes

    def admit(self, router: int) -> bool:
        """Admit a router now if a slot is free or the budget allows a new one; otherwise
        queue it (its batches are held) and return False."""
        with self.lock:
            if router in self.by_router:
                return True
            slot = self._take_slot()
            if slot is None:
                if router not in self.waiting:
                    self.waiting.append(router)
                self.refused += 1
                return False
            self._bind(slot, router)
            return True

    def _take_slot(self):
        if self.free:
            return self.free.pop()
        if len(self.slots) >= self.max_slots:
            return None
        s = Slot(self.params, len(self.slots))
        self.slots.append(s)
        return s

    def _bind(self, slot: Slot, router: int):
        slot.router = router
        self.by_router[router] = slot
        # a reused sketch restarts at the serving clock
        if self.slice_no and slot.sketch.cur < self.slice_no:
            slot.sketch.advance(self.slice_no)
        for pk, t in self.held.pop(router, []):
            self.pending.append((slot, pk, t))

    def release(self, router: int):
        """Router leaves: its slot is reset on the serving stream and reused."""
        with self.lock:
            slot = self.by_router.pop(router, None)
            if slot is None:
                return
            self.pending = [b for b in self.pending if b[0] is not slot]
            with torch.cuda.stream(self.stream):
                slot.sketch.reset()
            slot.router = None
            self.free.append(slot)
            while self.waiting and self.free:
                self._bind(self._take_slot(), self.waiting.popleft())

    # ---------------------------------------------------------------- arrivals
    def submit(self, router: int, pkts: torch.Tensor, arrival: float | None = None):
        """Queue a device-resident batch (n x 2 int32) for the next slice launch."""
        t = now() if arrival is None else arrival
        with self.lock:
            slot = self.by_router.get(router)
            if slot is None:
                self.held[router].append((pkts, t))
            else:
                self.pending.append((slot, pkts, t))

    # ---------------------------------------------------------------- slices
    def run_slice(self):
        """Launch one slice: batched ingest of everything pending, then every resident
        router's scan, as one captured graph on the serving stream."""
        while len(self.inflight) >= self.depth:
            self.collect(block=True, limit=1)
        with self.lock:
            batch, self.pending = self.pending, []
            active = [(s, s.router) for s in self.slots if s.router is not None]
        st = self.stream
        if self.slice_no + 1 > sps.SLICE_MAX:
            self._rebase(self.slice_no - self.window)
        self.slice_no += 1
        s_no = self.slice_no
        abs_no = s_no + self.slice_base
        par = abs_no % self.depth
        with torch.cuda.stream(st):
            for s, _ in active:
                if s.sketch.cur < s_no:
                    s.sketch.advance(s_no)
            t0 = now()
            if self.use_graph:
                sps.sps_graph_begin(st)
            try:
                if batch:
                    sps.sps_ingest_batched([b[0].sketch.h for b in batch], [b[1] for b in batch],
                                           s_no, st)
                for s, _ in active:
                    sps.sps_scan_async(s.sketch.h, self.window, self.threshold,
                                       self.res[par, s.index], self.cap, self.info[par, s.index],
                                       st)
            finally:
                if self.use_graph:
                    t1 = now()
                    # the buffer's previous slice has been collected, so its graph is idle
                    if self.graphs[par] is None:
                        self.graphs[par] = sps.sps_graph_end(st)
                        kind = "instantiate"
                    else:
                        kind = "update" if sps.sps_graph_end_update(self.graphs[par], st) \
                            else "instantiate"
                    self.host_ms["capture"].append(1e3 * (t1 - t0))
                    self.host_ms[kind].append(1e3 * (now() - t1))
            if self.use_graph:
                sps.sps_graph_launch(self.graphs[par], st)
            t_gpu = np.zeros(1, dtype=np.float64)  # written by the host notification
            sps.sps_stream_host_time(t_gpu, st)
            done = torch.cuda.Event()
            done.record(st)
        per_router = collections.defaultdict(list)
        for slot, p, t in batch:
            per_router[slot.router].append((p.shape[0], t))
        self.inflight.append((abs_no, done, t_gpu, active, per_router))

    def _rebase(self, offset: int):
        """Shift the time base of every sketch that holds stamps by `offset` (stream-ordered
        behind the slices already launched).  Reset slots (current slice 0) hold none."""
        with torch.cuda.stream(self.stream):
            for slot in self.slots:
                if slot.sketch.cur >= offset:
                    slot.sketch.rebase(offset, self.stream)
        self.slice_no -= offset
        self.slice_base += offset
        self.rebases += 1

    def collect(self, block: bool = False, limit: int = 1 << 30):
        """Turn finished slices into reports, in slice order (block: wait for them)."""
        while self.inflight and limit > 0:
            s_no, done, t_gpu, active, per_router = self.inflight[0]
            if not block and not done.query():
                return
            done.synchronize()
            self.inflight.popleft()
            limit -= 1
            par = s_no % self.depth
            info = self.info[par].cpu().numpy()
            res = self.res[par].cpu().numpy()
            t_done, t_rep = float(t_gpu[0]), now()
            for slot, router in active:
                kept = int(info[slot.index, sps.INFO_KEPT])
                flags = int(info[slot.index, sps.INFO_FLAGS])
                n = min(kept, self.cap)
                r = res[slot.index].view(sps.RESULT_DTYPE)[:n].copy()
                b = per_router.get(router, [])
                self.reports.append(Report(router, s_no, r, len(b), sum(x[0] for x in b),
                                           [t_done - t for _, t in b], flags, kept,
                                           [t_rep - t for _, t in b]))
                if flags:
                    self.incomplete += 1

    def close(self):
        """Collect launched slices and free the graphs and sketches."""
        try:
            self.collect(block=True)
        finally:
            for g in self.graphs:
                if g is not None:
                    sps.sps_graph_destroy(g)
            self.graphs = [None] * self.depth
            for s in self.slots:
                s.sketch.close()

    def autotune(self, batches, slice_: int = 1):
        """Pick the batched-ingest launch shape on a representative set of batches
        [(router, pkts)] of resident routers (sps_autotune_ingest), then reset those routers'
        sketches, so serving starts from empty sketches with the tuned shape."""
        with self.lock:
            slots = [self.by_router[r] for r, _ in batches]
        best, ms = sps.sps_autotune_ingest([s.sketch.h for s in slots], [p for _, p in batches],
                                           slice_, self.stream)
        for s in self.slots:
            sps.sps_set_tuning(s.sketch.h, **best)
        with torch.cuda.stream(self.stream):
            for s in {id(x): x for x in slots}.values():
                s.sketch.reset()
        self.stream.synchronize()
        return best, ms


def poisson_schedule(seed: int, rate_pkts: float, duration_s: float, n_routers: int,
                     lo: int = 4096, hi: int = 4 << 20):
    """Arrival times, routers and sizes of a Poisson batch process with log-uniform batch
    sizes in [lo, hi] and `rate_pkts` packets per second on average."""
    g = np.random.Generator(np.random.Philox(seed))
    mean_size = (hi - lo) / np.log(hi / lo)
    rate = rate_pkts / mean_size
    n = int(rate * duration_s * 1.2) + 16
    t = np.cumsum(g.exponential(1.0 / rate, n))
    t = t[t < duration_s]
    sizes = np.exp(g.uniform(np.log(lo), np.log(hi), len(t))).astype(np.int64)
    routers = g.integers(0, n_routers, len(t))
    return t, routers, sizes


def run_simulation(server: Server, pool: torch.Tensor, schedule, slice_s: float, n_slices: int,
                   seed: int = 1, departures: dict | None = None):
    """Real-time replay: an arrival thread submits the schedule's batches (slices of the
    device-resident packet pool) at their times; the main loop launches a slice every
    slice_s seconds and collects finished ones.  departures: {slice: [routers]} leaving after
    that slice.  Returns (wall seconds, packets submitted)."""
    t_arr, routers, sizes = schedule
    g = np.random.Generator(np.random.Philox(seed))
    offs = g.integers(0, pool.shape[0] - sizes.max(), len(sizes))
    t0 = now()
    stop = threading.Event()

    def arrivals():
        for i in range(len(t_arr)):
            if stop.is_set():
                return
            dt = t0 + t_arr[i] - now()
            if dt > 0:
                time.sleep(dt)
            o = int(offs[i])
            server.submit(int(routers[i]), pool[o:o + int(sizes[i])])

    th = threading.Thread(target=arrivals, daemon=True)
    th.start()
    for k in range(n_slices):
        target = t0 + (k + 1) * slice_s
        dt = target - now()
        if dt > 0:
            time.sleep(dt)
        server.run_slice()
        server.collect()
        if departures and (k + 1) in departures:
            for r in departures[k + 1]:
                server.release(r)
    stop.set()
    th.join()
    server.collect(block=True)
    wall = now() - t0
    return wall, int(sizes[t_arr < n_slices * slice_s].sum())
