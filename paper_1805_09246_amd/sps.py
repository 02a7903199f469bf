"""Thin ctypes binding of the sliding super point sketch library (include/sps.h).

Functions carry the C names and only marshal arguments: torch CUDA tensors become device
pointers, ``torch.cuda`` streams become hipStream_t handles, numpy arrays hold host data.
Every step of the method runs in the HIP kernels of ``libsps.so``; if the library is not
built this module raises instead of computing anything itself.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np
import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libsps.so")

SPS_OK, SPS_EINVAL, SPS_ESLICE, SPS_EMISMATCH = 0, -1, -2, -3
SPS_ENOMEM, SPS_ECAPACITY, SPS_EHIP, SPS_EBUDGET = -4, -5, -6, -7
F_SATURATED, F_LC_FALLBACK, F_MLP, F_NEAR, F_CLAMPLOW = 1, 2, 4, 8, 16
INFO_KEPT, INFO_CAND, INFO_FLAGS, INFO_HSE0, INFO_HSE1, INFO_WORDS = 0, 1, 2, 3, 4, 8
INFO_NODES_LO, INFO_NODES_HI = 5, 6
MLP_IN, MLP_HIDDEN = 10, 64
MLP_NOALLOC_MAX_N = 4096
MLP_PARAMS = MLP_HIDDEN * MLP_IN + MLP_HIDDEN + MLP_HIDDEN * MLP_HIDDEN + MLP_HIDDEN + MLP_HIDDEN + 1
HEADER_BYTES = 64

EXPORTS = [
    "sps_sketch_bytes", "sps_create", "sps_destroy", "sps_reset", "sps_ingest",
    "sps_ingest_batched", "sps_advance", "sps_merge", "sps_scan", "sps_scan_async",
    "sps_features", "sps_attach_mlp", "sps_state_bytes", "sps_export", "sps_import",
    "sps_current_slice", "sps_derived", "sps_debug_copy", "sps_sync", "sps_strerror",
    "sps_profile_enable", "sps_profile_read", "sps_probe_scatter", "sps_probe_stream",
    "sps_estimate_hosts", "sps_mlp_work_bytes", "sps_mlp_grad", "sps_mlp_adam",
    "sps_mlp_forward", "sps_get_tuning", "sps_set_tuning", "sps_autotune_ingest",
    "sps_graph_begin", "sps_graph_end", "sps_graph_launch", "sps_graph_destroy", "sps_rebase",
    "sps_mlp_grad_noalloc", "sps_probe_replay_record", "sps_probe_replay",
    "sps_graph_end_update", "sps_tuning_lookup", "sps_tuning_cache_save",
    "sps_tuning_cache_load", "sps_tuning_cache_clear", "sps_stream_host_time",
]
STAGES = ["ingest", "ingest_batched", "merge", "fill", "scan_reset", "scan_stats", "join",
          "estimate", "sort", "features", "probe", "mlp", "scan", "rebase", "scan_rows"]
SLICE_MAX = 65534


class sps_tuning(C.Structure):
    _fields_ = [("blocks_per_cu", C.c_uint32), ("batch_tile", C.c_uint32),
                ("host_classes", C.c_uint32), ("scan_overlap", C.c_uint32)]


class SpsError(RuntimeError):
    def __init__(self, code: int, where: str):
        self.code = code
        super().__init__(f"{where}: {strerror(code)} ({code})")


class sps_params(C.Structure):
    _fields_ = [("q", C.c_uint32), ("r", C.c_uint32), ("delta", C.c_uint32), ("eta", C.c_uint32),
                ("qp", C.c_uint32), ("rp", C.c_uint32), ("etap", C.c_uint32),
                ("deltap", C.c_uint32), ("theta", C.c_uint32), ("anet_side", C.c_uint32),
                ("seed", C.c_uint64), ("cand_cap", C.c_uint32), ("mode", C.c_uint32),
                ("row_counts", C.c_uint32)]


RESULT_DTYPE = np.dtype([("host", "<u4"), ("live", "<u4"), ("flags", "<u4"), ("pad", "<u4"),
                         ("estimate", "<f8")])
assert RESULT_DTYPE.itemsize == 24

_lib = None


def lib():
    """Load libsps.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with __graft_entry__.build()")
        L = C.CDLL(LIB_PATH)
        vp, u32, u64, sz, i32 = C.c_void_p, C.c_uint32, C.c_uint64, C.c_size_t, C.c_int
        P = C.POINTER
        sig = {
            "sps_sketch_bytes": [P(sps_params), P(sz)],
            "sps_create": [P(sps_params), vp, sz, P(vp)],
            "sps_destroy": [vp],
            "sps_reset": [vp, vp],
            "sps_ingest": [vp, vp, sz, u32, vp],
            "sps_ingest_batched": [P(vp), P(vp), P(sz), u32, u32, vp],
            "sps_advance": [vp, u32],
            "sps_rebase": [vp, u32, vp],
            "sps_merge": [vp, P(vp), u32, vp],
            "sps_scan": [vp, u32, C.c_double, vp, sz, P(sz), vp],
            "sps_scan_async": [vp, u32, C.c_double, vp, sz, vp, vp],
            "sps_features": [vp, vp, sz, u32, vp, vp],
            "sps_attach_mlp": [vp, vp, vp, vp, u32, C.c_double],
            "sps_estimate_hosts": [vp, vp, sz, u32, vp, vp],
            "sps_mlp_work_bytes": [sz, P(sz)],
            "sps_mlp_grad": [vp, vp, vp, vp, sz, u32, vp, vp, vp, vp],
            "sps_mlp_grad_noalloc": [vp, vp, vp, vp, sz, u32, vp, vp, vp],
            "sps_mlp_adam": [vp, vp, vp, vp, u32, C.c_float, C.c_double, C.c_double, C.c_float, vp],
            "sps_mlp_forward": [vp, vp, sz, u32, C.c_int, vp, vp],
            "sps_get_tuning": [vp, P(sps_tuning)],
            "sps_set_tuning": [vp, P(sps_tuning)],
            "sps_autotune_ingest": [P(vp), P(vp), P(sz), u32, u32, vp, P(sps_tuning), vp, u32],
            "sps_tuning_lookup": [C.c_char_p, P(sps_params), u32, P(sps_tuning), P(i32)],
            "sps_tuning_cache_save": [C.c_char_p],
            "sps_tuning_cache_load": [C.c_char_p],
            "sps_tuning_cache_clear": [],
            "sps_stream_host_time": [vp, vp],
            "sps_graph_begin": [vp],
            "sps_graph_end": [vp, P(vp)],
            "sps_graph_launch": [vp, vp],
            "sps_graph_end_update": [vp, vp, P(i32)],
            "sps_graph_destroy": [vp],
            "sps_state_bytes": [vp, P(sz)],
            "sps_export": [vp, vp, sz, vp],
            "sps_import": [vp, vp, sz, vp],
            "sps_current_slice": [vp, P(u32)],
            "sps_derived": [vp, P(u32), P(u32), P(u64)],
            "sps_debug_copy": [vp, i32, vp, sz, P(sz), vp],
            "sps_sync": [vp],
            "sps_profile_enable": [u32],
            "sps_profile_read": [vp, vp, i32],
            "sps_probe_scatter": [vp, u64, u64, u32, C.c_uint16, vp],
            "sps_probe_stream": [vp, u64, vp, vp],
            "sps_probe_replay_record": [vp, vp, sz, vp, sz, P(u64), vp],
            "sps_probe_replay": [vp, vp, P(u64), C.c_uint16, vp],
        }
        for name, args in sig.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = i32
        L.sps_strerror.argtypes = [i32]
        L.sps_strerror.restype = C.c_char_p
        _lib = L
    return _lib


def strerror(code: int) -> str:
    return lib().sps_strerror(code).decode()


def _check(rc: int, where: str):
    if rc != SPS_OK:
        raise SpsError(rc, where)


def _stream(stream):
    if stream is None:
        stream = torch.cuda.current_stream()
    return C.c_void_p(stream.cuda_stream)


def _dptr(t: torch.Tensor):
    assert t.is_cuda and t.is_contiguous(), "device tensor expected"
    return C.c_void_p(t.data_ptr())


def make_params(d: dict) -> sps_params:
    return sps_params(**{k: int(d.get(k, 0)) for k, _ in sps_params._fields_})


# ---------------------------------------------------------------- C functions, same names
def sps_sketch_bytes(params: dict) -> int:
    n = C.c_size_t(0)
    p = make_params(params)
    _check(lib().sps_sketch_bytes(C.byref(p), C.byref(n)), "sps_sketch_bytes")
    return n.value


def sps_create(params: dict, dev_mem: torch.Tensor | None = None):
    p = make_params(params)
    h = C.c_void_p(0)
    if dev_mem is None:
        rc = lib().sps_create(C.byref(p), None, 0, C.byref(h))
    else:
        rc = lib().sps_create(C.byref(p), _dptr(dev_mem), dev_mem.numel() * dev_mem.element_size(),
                              C.byref(h))
    _check(rc, "sps_create")
    return h


def sps_destroy(h):
    _check(lib().sps_destroy(h), "sps_destroy")


def sps_reset(h, stream=None):
    _check(lib().sps_reset(h, _stream(stream)), "sps_reset")


def _check_pairs(pkts: torch.Tensor, where: str) -> int:
    """Number of pairs in an (n, 2) tensor of 32-bit (src, dst) values on the device; raises
    before any launch for any other shape, width or placement."""
    if not (pkts.dim() == 2 and pkts.shape[1] == 2 and pkts.element_size() == 4):
        raise ValueError(f"{where}: packets must be an (n, 2) 32-bit tensor, got "
                         f"{tuple(pkts.shape)} of {pkts.dtype}")
    n = int(pkts.shape[0])
    if n and not (pkts.is_cuda and pkts.is_contiguous()):
        raise ValueError(f"{where}: packets must be a contiguous device tensor")
    return n


def sps_ingest(h, pkts: torch.Tensor, slice_: int, stream=None):
    """pkts: (n, 2) 32-bit device tensor of (src, dst) pairs."""
    n = _check_pairs(pkts, "sps_ingest")
    ptr = _dptr(pkts) if n else None
    _check(lib().sps_ingest(h, ptr, n, slice_, _stream(stream)), "sps_ingest")


def _batch_arrays(hs, pkts_list, where):
    m = len(hs)
    if m != len(pkts_list) or m == 0:
        raise ValueError(f"{where}: {m} sketches for {len(pkts_list)} packet batches")
    ns = [_check_pairs(p, where) for p in pkts_list]
    harr = (C.c_void_p * m)(*[h.value for h in hs])
    parr = (C.c_void_p * m)(*[(p.data_ptr() if n else 0) for p, n in zip(pkts_list, ns)])
    narr = (C.c_size_t * m)(*ns)
    return m, harr, parr, narr


def sps_ingest_batched(hs, pkts_list, slice_: int, stream=None):
    m, harr, parr, narr = _batch_arrays(hs, pkts_list, "sps_ingest_batched")
    _check(lib().sps_ingest_batched(harr, parr, narr, m, slice_, _stream(stream)),
           "sps_ingest_batched")


def sps_advance(h, slice_: int):
    _check(lib().sps_advance(h, slice_), "sps_advance")


def sps_rebase(h, offset: int, stream=None):
    _check(lib().sps_rebase(h, offset, _stream(stream)), "sps_rebase")


def sps_merge(dst, srcs, stream=None):
    arr = (C.c_void_p * max(1, len(srcs)))(*[s.value for s in srcs])
    _check(lib().sps_merge(dst, arr, len(srcs), _stream(stream)), "sps_merge")


def sps_scan(h, window: int, threshold: float, cap: int = 1 << 16, stream=None) -> np.ndarray:
    out = np.zeros(cap, dtype=RESULT_DTYPE)
    n = C.c_size_t(0)
    rc = lib().sps_scan(h, window, threshold, out.ctypes.data_as(C.c_void_p), cap, C.byref(n),
                        _stream(stream))
    if rc == SPS_ECAPACITY:
        raise SpsError(rc, f"sps_scan (required {n.value})")
    _check(rc, "sps_scan")
    return out[: n.value].copy()


def sps_scan_async(h, window: int, threshold: float, d_out: torch.Tensor, cap: int,
                   d_info: torch.Tensor, stream=None):
    """d_out: device buffer of >= cap * 24 bytes; d_info: device buffer of >= 8 x 4 bytes."""
    assert d_out.numel() * d_out.element_size() >= cap * 24
    assert d_info.numel() * d_info.element_size() >= INFO_WORDS * 4
    _check(lib().sps_scan_async(h, window, threshold, _dptr(d_out), cap, _dptr(d_info),
                                _stream(stream)), "sps_scan_async")


def sps_features(h, d_hosts: torch.Tensor, window: int, d_x: torch.Tensor, stream=None):
    n = d_hosts.numel()
    assert d_x.numel() >= n * window and d_x.element_size() == 4 and d_hosts.element_size() == 4
    _check(lib().sps_features(h, _dptr(d_hosts) if n else None, n, window,
                              _dptr(d_x) if n else None, _stream(stream)), "sps_features")


def sps_attach_mlp(h, d_weights: torch.Tensor | None, feat_lo=None, feat_hi=None,
                   min_live: int = 0, max_card: float = 1e6):
    if d_weights is None:
        _check(lib().sps_attach_mlp(h, None, None, None, 0, 0.0), "sps_attach_mlp")
        return
    assert d_weights.dtype == torch.float32 and d_weights.numel() == MLP_PARAMS
    lo = np.ascontiguousarray(feat_lo, dtype=np.float32)
    hi = np.ascontiguousarray(feat_hi, dtype=np.float32)
    _check(lib().sps_attach_mlp(h, _dptr(d_weights), lo.ctypes.data_as(C.c_void_p),
                                hi.ctypes.data_as(C.c_void_p), int(min_live), max_card),
           "sps_attach_mlp")


def sps_estimate_hosts(h, d_hosts: torch.Tensor, window: int, stream=None) -> torch.Tensor:
    """Returns a (n * 24)-byte uint8 device tensor of sps_result records (input order)."""
    n = d_hosts.numel()
    out = torch.zeros(max(1, n) * 24, dtype=torch.uint8, device=d_hosts.device)
    _check(lib().sps_estimate_hosts(h, _dptr(d_hosts) if n else None, n, window, _dptr(out),
                                    _stream(stream)), "sps_estimate_hosts")
    return out


def results_to_numpy(t: torch.Tensor, n: int) -> np.ndarray:
    return t.cpu().numpy().view(RESULT_DTYPE)[:n]


def sps_mlp_work_bytes(n: int) -> int:
    b = C.c_size_t(0)
    _check(lib().sps_mlp_work_bytes(n, C.byref(b)), "sps_mlp_work_bytes")
    return b.value


def sps_mlp_grad(d_w, d_feat, d_target, d_idx, n: int, etap: int, d_work, d_grad, d_loss=None,
                 stream=None):
    _check(lib().sps_mlp_grad(_dptr(d_w), _dptr(d_feat), _dptr(d_target),
                              _dptr(d_idx) if d_idx is not None else None, n, etap,
                              _dptr(d_work), _dptr(d_grad),
                              _dptr(d_loss) if d_loss is not None else None, _stream(stream)),
           "sps_mlp_grad")


def sps_mlp_grad_noalloc(d_w, d_feat, d_target, d_idx, n: int, etap: int, d_grad, d_loss=None,
                         stream=None):
    _check(lib().sps_mlp_grad_noalloc(_dptr(d_w), _dptr(d_feat), _dptr(d_target),
                                      _dptr(d_idx) if d_idx is not None else None, n, etap,
                                      _dptr(d_grad),
                                      _dptr(d_loss) if d_loss is not None else None,
                                      _stream(stream)),
           "sps_mlp_grad_noalloc")


def sps_mlp_adam(d_w, d_m, d_v, d_grad, step: int, lr: float, beta1=0.9, beta2=0.999, eps=1e-8,
                 stream=None):
    _check(lib().sps_mlp_adam(_dptr(d_w), _dptr(d_m), _dptr(d_v), _dptr(d_grad), step, lr, beta1,
                              beta2, eps, _stream(stream)), "sps_mlp_adam")


def sps_mlp_forward(d_w, d_feat, n: int, etap: int, bf16: bool, d_y, stream=None):
    _check(lib().sps_mlp_forward(_dptr(d_w), _dptr(d_feat) if n else None, n, etap,
                                 1 if bf16 else 0, _dptr(d_y) if n else None, _stream(stream)),
           "sps_mlp_forward")


def sps_state_bytes(h) -> int:
    n = C.c_size_t(0)
    _check(lib().sps_state_bytes(h, C.byref(n)), "sps_state_bytes")
    return n.value


def sps_export(h, stream=None) -> np.ndarray:
    buf = np.zeros(sps_state_bytes(h), dtype=np.uint8)
    _check(lib().sps_export(h, buf.ctypes.data_as(C.c_void_p), buf.nbytes, _stream(stream)),
           "sps_export")
    return buf


def sps_import(h, buf: np.ndarray, stream=None):
    buf = np.ascontiguousarray(buf, dtype=np.uint8)
    _check(lib().sps_import(h, buf.ctypes.data_as(C.c_void_p), buf.nbytes, _stream(stream)),
           "sps_import")


def sps_current_slice(h) -> int:
    v = C.c_uint32(0)
    _check(lib().sps_current_slice(h, C.byref(v)), "sps_current_slice")
    return v.value


def sps_derived(h):
    tau, cut, rl = C.c_uint32(0), C.c_uint32(0), C.c_uint64(0)
    _check(lib().sps_derived(h, C.byref(tau), C.byref(cut), C.byref(rl)), "sps_derived")
    return tau.value, cut.value, rl.value


def sps_debug_copy(h, which: int, stream=None) -> np.ndarray:
    size = C.c_size_t(0)
    _check(lib().sps_debug_copy(h, which, None, 0, C.byref(size), _stream(stream)),
           "sps_debug_copy")
    buf = np.zeros(size.value, dtype=np.uint8)
    if size.value:
        _check(lib().sps_debug_copy(h, which, buf.ctypes.data_as(C.c_void_p), buf.nbytes,
                                    C.byref(size), _stream(stream)), "sps_debug_copy")
    return buf


def sps_sync(stream=None):
    _check(lib().sps_sync(_stream(stream)), "sps_sync")


def sps_strerror(code: int) -> str:
    return strerror(code)


def sps_profile_enable(on, stages=None):
    """on: False disables; True records every stage, or only the named `stages`."""
    if not on:
        mask = 0
    elif stages is None:
        mask = 0xFFFFFFFF
    else:
        mask = 0
        for st in stages:
            mask |= 1 << STAGES.index(st)
    _check(lib().sps_profile_enable(mask), "sps_profile_enable")


def sps_profile_read() -> dict:
    """{stage name: (total ms, launches)} since the last read (synchronizes)."""
    n = len(STAGES)
    ms = np.zeros(n, dtype=np.float64)
    cnt = np.zeros(n, dtype=np.uint32)
    _check(lib().sps_profile_read(ms.ctypes.data_as(C.c_void_p), cnt.ctypes.data_as(C.c_void_p),
                                  n), "sps_profile_read")
    return {STAGES[i]: (float(ms[i]), int(cnt[i])) for i in range(n)}


def sps_probe_scatter(d_cells: torch.Tensor, n_stores: int, seed: int, value: int, stream=None):
    assert d_cells.element_size() == 2
    _check(lib().sps_probe_scatter(_dptr(d_cells), d_cells.numel(), n_stores, seed, value,
                                   _stream(stream)), "sps_probe_scatter")


def sps_probe_replay_record(h, pkts: torch.Tensor, stream=None):
    """(cells, class offsets): the cells sps_ingest(h, pkts) writes, grouped by host class."""
    n = _check_pairs(pkts, "sps_probe_replay_record")
    off = (C.c_uint64 * 9)()
    rc = lib().sps_probe_replay_record(h, _dptr(pkts) if n else None, n, None, 0, off,
                                       _stream(stream))
    if rc not in (SPS_OK, SPS_ECAPACITY):
        _check(rc, "sps_probe_replay_record")
    cells = torch.empty(max(1, off[8]), dtype=torch.int32, device=pkts.device)
    _check(lib().sps_probe_replay_record(h, _dptr(pkts) if n else None, n, _dptr(cells),
                                         cells.numel(), off, _stream(stream)),
           "sps_probe_replay_record")
    return cells, (C.c_uint64 * 9)(*off)


def sps_probe_replay(h, cells: torch.Tensor, class_off, value: int, stream=None):
    _check(lib().sps_probe_replay(h, _dptr(cells), class_off, value, _stream(stream)),
           "sps_probe_replay")


def sps_probe_stream(d_buf: torch.Tensor, d_sum: torch.Tensor, stream=None):
    nbytes = d_buf.numel() * d_buf.element_size()
    _check(lib().sps_probe_stream(_dptr(d_buf), nbytes, _dptr(d_sum), _stream(stream)),
           "sps_probe_stream")


def _tuning_dict(t) -> dict:
    """The ingest's launch shape (what the tuner and the tuning cache hold)."""
    return {"blocks_per_cu": t.blocks_per_cu, "batch_tile": t.batch_tile,
            "host_classes": t.host_classes}


def sps_get_scan_overlap(h) -> bool:
    t = sps_tuning()
    _check(lib().sps_get_tuning(h, C.byref(t)), "sps_get_tuning")
    return t.scan_overlap == 1


def sps_get_tuning(h) -> dict:
    t = sps_tuning()
    _check(lib().sps_get_tuning(h, C.byref(t)), "sps_get_tuning")
    return _tuning_dict(t)


def sps_set_tuning(h, blocks_per_cu: int = 0, batch_tile: int = 0, host_classes: int = 0,
                   scan_overlap: int = 0):
    t = sps_tuning(blocks_per_cu, batch_tile, host_classes, scan_overlap)
    _check(lib().sps_set_tuning(h, C.byref(t)), "sps_set_tuning")


AUTOTUNE_CANDIDATES_SINGLE, AUTOTUNE_CANDIDATES_BATCHED = 12, 48


def sps_autotune_ingest(hs, pkts_list, slice_: int, stream=None):
    """Returns (best tuning dict, list of candidate times in ms)."""
    m, harr, parr, narr = _batch_arrays(hs, pkts_list, "sps_autotune_ingest")
    best = sps_tuning()
    ms = np.zeros(64, dtype=np.float32)
    _check(lib().sps_autotune_ingest(harr, parr, narr, m, slice_, _stream(stream), C.byref(best),
                                     ms.ctypes.data_as(C.c_void_p), 64), "sps_autotune_ingest")
    n = AUTOTUNE_CANDIDATES_SINGLE if m == 1 else AUTOTUNE_CANDIDATES_BATCHED
    return _tuning_dict(best), ms[:n].tolist()


def sps_tuning_lookup(params: dict, batched: bool, arch: str | None = None):
    """The cached tuning dict for (arch, sketch shape, batched), or None."""
    p = make_params(params)
    t = sps_tuning()
    found = C.c_int(0)
    _check(lib().sps_tuning_lookup(arch.encode() if arch is not None else None, C.byref(p),
                                   1 if batched else 0, C.byref(t), C.byref(found)),
           "sps_tuning_lookup")
    return _tuning_dict(t) if found.value else None


def sps_tuning_cache_save(path: str):
    _check(lib().sps_tuning_cache_save(path.encode()), "sps_tuning_cache_save")


def sps_tuning_cache_load(path: str):
    _check(lib().sps_tuning_cache_load(path.encode()), "sps_tuning_cache_load")


def sps_tuning_cache_clear():
    _check(lib().sps_tuning_cache_clear(), "sps_tuning_cache_clear")


def sps_graph_begin(stream=None):
    _check(lib().sps_graph_begin(_stream(stream)), "sps_graph_begin")


def sps_graph_end(stream=None):
    g = C.c_void_p(0)
    _check(lib().sps_graph_end(_stream(stream), C.byref(g)), "sps_graph_end")
    return g


def sps_graph_end_update(g, stream=None) -> bool:
    """End the capture and update g with it; True when updated in place."""
    u = C.c_int(0)
    _check(lib().sps_graph_end_update(_stream(stream), g, C.byref(u)), "sps_graph_end_update")
    return bool(u.value)


def sps_stream_host_time(h_time: np.ndarray, stream=None):
    """h_time: float64 numpy array; element 0 receives the host CLOCK_MONOTONIC seconds when
    the stream reaches this point.  The caller keeps the array alive until then."""
    assert h_time.dtype == np.float64 and h_time.flags.c_contiguous and h_time.size >= 1
    _check(lib().sps_stream_host_time(h_time.ctypes.data_as(C.c_void_p), _stream(stream)),
           "sps_stream_host_time")


def sps_graph_launch(g, stream=None):
    _check(lib().sps_graph_launch(g, _stream(stream)), "sps_graph_launch")


def sps_graph_destroy(g):
    _check(lib().sps_graph_destroy(g), "sps_graph_destroy")


# ---------------------------------------------------------------- convenience owner
class Sketch:
    """Owns a sketch and the torch device block it lives in."""

    def __init__(self, params: dict, device: str = "cuda"):
        self.params = dict(params)
        self.nbytes = sps_sketch_bytes(params)
        self.mem = torch.empty(self.nbytes, dtype=torch.uint8, device=device)
        self.h = sps_create(params, self.mem)

    def close(self):
        if getattr(self, "h", None) is not None:
            sps_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # thin forwards
    def reset(self, stream=None):
        sps_reset(self.h, stream)

    def ingest(self, pkts, slice_, stream=None):
        sps_ingest(self.h, pkts, slice_, stream)

    def advance(self, slice_):
        sps_advance(self.h, slice_)

    def rebase(self, offset, stream=None):
        sps_rebase(self.h, offset, stream)

    def merge(self, srcs, stream=None):
        sps_merge(self.h, [s.h for s in srcs], stream)

    def scan(self, window, threshold, cap=1 << 16, stream=None):
        return sps_scan(self.h, window, threshold, cap, stream)

    def features(self, hosts: torch.Tensor, window: int, stream=None) -> torch.Tensor:
        x = torch.zeros((hosts.numel(), window), dtype=torch.int32, device=hosts.device)
        sps_features(self.h, hosts, window, x, stream)
        return x

    @property
    def cur(self):
        return sps_current_slice(self.h)

    def derived(self):
        return sps_derived(self.h)

    def export(self, stream=None) -> np.ndarray:
        return sps_export(self.h, stream)

    def import_(self, buf, stream=None):
        sps_import(self.h, buf, stream)

    def state(self, stream=None):
        """(SRE u16 (r, 2^q, eta), SLE array u16 (r', L')) from a bit-exact dump."""
        return split_dump(self.export(stream), self.params)


MODE_SLIDING, MODE_DISCRETE = 0, 1


def split_dump(buf: np.ndarray, params: dict):
    """Sliding mode: (u16 SRE (r, 2^q, eta), u16 SLE array (r', L')).  Discrete mode: the
    same shapes as uint8 0/1 arrays of the recorder bits."""
    p = params
    n_sre = (p["r"] << p["q"]) * p["eta"]
    row_len = (1 << p["qp"]) * p["deltap"] + p["etap"] - p["deltap"]
    if p.get("mode", 0) == MODE_DISCRETE:
        body = buf[HEADER_BYTES:]
        sre = np.unpackbits(body[:n_sre // 8], bitorder="little").reshape(
            p["r"], 1 << p["q"], p["eta"])
        rw = (row_len + 31) // 32 * 4
        rows = body[n_sre // 8:n_sre // 8 + p["rp"] * rw].reshape(p["rp"], rw)
        slea = np.unpackbits(rows, axis=1, bitorder="little")[:, :row_len]
        return sre, slea
    body = buf[HEADER_BYTES:].view(np.uint16)
    sre = body[:n_sre].reshape(p["r"], 1 << p["q"], p["eta"])
    slea = body[n_sre:n_sre + p["rp"] * row_len].reshape(p["rp"], row_len)
    return sre, slea
