"""CPU oracle for the sliding super point sketch -- TEST INFRASTRUCTURE ONLY.

Only the test suite, the smoke check and the benchmark's CPU-baseline leg may import this
package.  The product library never loads it and shares no code with it.

Parts:
  * ``OracleSketch``: bit-exact SRE / SLE arrays, ingest (Alg. 3, Alg. 6), merge (Alg. 2,
    Alg. 7), k-weights and hot SREs (Sec. 3.2-3.3, Def. 4), candidate recovery (the plain
    definition by exhaustive search, and the paper's tuple growing of Alg. 4-5), estimate
    and filter (Alg. 8, Eq. 9, Eq. 12) -- all in ``sps_oracle.c``, wrapped here with ctypes.
  * ``truth``: exact per-host distinct-peer counts over a sliding window (Def. 1-2).
  * ``mlp``: fp64 forward / backward / Adam of the learned cardinality estimator.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liboracle.so")

F_SATURATED, F_NEAR, F_CLAMPLOW = 1, 8, 16


class _Params(C.Structure):
    _fields_ = [("q", C.c_uint32), ("r", C.c_uint32), ("delta", C.c_uint32), ("eta", C.c_uint32),
                ("qp", C.c_uint32), ("rp", C.c_uint32), ("etap", C.c_uint32),
                ("deltap", C.c_uint32), ("theta", C.c_uint32), ("anet_side", C.c_uint32),
                ("seed", C.c_uint64)]


RESULT_DTYPE = np.dtype([("host", "<u4"), ("live", "<u4"), ("flags", "<u4"), ("pad", "<u4"),
                         ("estimate", "<f8")])

_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            from . import build
            build.build()
        L = C.CDLL(LIB_PATH)
        P = C.POINTER
        vp = C.c_void_p
        L.or_create.restype = vp
        L.or_create.argtypes = [P(_Params)]
        L.or_destroy.argtypes = [vp]
        L.or_check_params.argtypes = [P(_Params)]
        for n in ("or_get_tau", "or_get_hot_cut", "or_get_cur"):
            getattr(L, n).restype = C.c_uint32
            getattr(L, n).argtypes = [vp]
        for n in ("or_get_row_len", "or_sre_cells", "or_slea_cells"):
            getattr(L, n).restype = C.c_uint64
            getattr(L, n).argtypes = [vp]
        L.or_sre_ptr.restype = vp
        L.or_sre_ptr.argtypes = [vp]
        L.or_slea_ptr.restype = vp
        L.or_slea_ptr.argtypes = [vp]
        L.or_lsb.restype = C.c_uint32
        L.or_lsb.argtypes = [C.c_uint32]
        L.or_tau.restype = C.c_uint32
        L.or_tau.argtypes = [C.c_uint32, C.c_uint32]
        L.or_hot_cut.restype = C.c_uint32
        L.or_hot_cut.argtypes = [C.c_uint32]
        L.or_row_len.restype = C.c_uint64
        L.or_row_len.argtypes = [C.c_uint32] * 3
        L.or_mrr.restype = C.c_double
        L.or_mrr.argtypes = [C.c_uint32] * 3
        L.or_hash.restype = C.c_uint32
        L.or_hash.argtypes = [vp, C.c_uint32, C.c_uint32, C.c_uint32]
        L.or_fmix32_export.restype = C.c_uint32
        L.or_fmix32_export.argtypes = [C.c_uint32]
        L.or_splitmix64_export.restype = C.c_uint64
        L.or_splitmix64_export.argtypes = [C.c_uint64]
        L.or_set_slice.argtypes = [vp, C.c_uint32]
        L.or_ingest.argtypes = [vp, vp, C.c_uint64, C.c_uint32]
        L.or_ingest_threads.argtypes = [vp, vp, C.c_uint64, C.c_uint32, C.c_uint32]
        L.or_merge.argtypes = [vp, P(vp), C.c_uint32]
        L.or_rebase.argtypes = [vp, C.c_uint32]
        L.or_row_live.argtypes = [vp, C.c_uint32, vp]
        L.or_hot.argtypes = [vp, C.c_uint32, vp]
        L.or_join_brute.restype = C.c_int64
        L.or_join_brute.argtypes = [vp, vp, vp, C.c_uint64, C.c_uint32]
        L.or_join_tuples.restype = C.c_int64
        L.or_join_tuples.argtypes = [vp, vp, vp, C.c_uint64, C.c_uint64, vp]
        L.or_features.argtypes = [vp, C.c_uint32, vp, C.c_uint64, vp]
        L.or_estimate_one.restype = C.c_double
        L.or_estimate_one.argtypes = [vp, C.c_uint32, vp, C.c_double, P(C.c_uint32)]
        L.or_estimate_filter.restype = C.c_int64
        L.or_estimate_filter.argtypes = [vp, C.c_uint32, C.c_double, vp, C.c_uint64, vp,
                                         C.c_uint64]
        L.or_scan.restype = C.c_int64
        L.or_scan.argtypes = [vp, C.c_uint32, C.c_double, vp, C.c_uint64, vp, C.c_uint64,
                              P(C.c_uint64), C.c_uint32]
        _lib = L
    return _lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(C.c_void_p)


def lsb(v: int) -> int:
    return int(lib().or_lsb(v))


def tau(theta: int, eta: int) -> int:
    return int(lib().or_tau(theta, eta))


def hot_cut(eta: int) -> int:
    return int(lib().or_hot_cut(eta))


def row_len(qp: int, etap: int, deltap: int) -> int:
    return int(lib().or_row_len(qp, etap, deltap))


def mrr(qp: int, etap: int, deltap: int) -> float:
    return float(lib().or_mrr(qp, etap, deltap))


def fmix32(h: int) -> int:
    return int(lib().or_fmix32_export(h))


def splitmix64_next(state: int) -> int:
    """Output of SplitMix64 after one step from `state`."""
    return int(lib().or_splitmix64_export(state))


def default_threads() -> int:
    return max(1, min(16, os.cpu_count() or 1))


class OracleSketch:
    """Bit-exact CPU sketch.  ``params``: dict with the sps_params field names."""

    H1, H2, H3, RHFG, LH = range(5)

    def __init__(self, params: dict):
        self.params = dict(params)
        self._p = _Params(**{k: params[k] for k, _ in _Params._fields_})
        h = lib().or_create(C.byref(self._p))
        if not h:
            raise ValueError(f"oracle rejected params {params}")
        self._h = C.c_void_p(h)
        L = lib()
        self.tau = int(L.or_get_tau(self._h))
        self.hot_cut = int(L.or_get_hot_cut(self._h))
        self.row_len = int(L.or_get_row_len(self._h))
        self._n_sre = int(L.or_sre_cells(self._h))
        self._n_slea = int(L.or_slea_cells(self._h))

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and _lib is not None:
            _lib.or_destroy(h)
            self._h = None

    # --- state --------------------------------------------------------------------------
    @property
    def cur(self) -> int:
        return int(lib().or_get_cur(self._h))

    def sre(self) -> np.ndarray:
        """View of the SRE stamps, shape (r, 2^q, eta)."""
        p = self.params
        buf = (C.c_uint16 * self._n_sre).from_address(lib().or_sre_ptr(self._h))
        return np.frombuffer(buf, dtype=np.uint16).reshape(p["r"], 1 << p["q"], p["eta"])

    def slea(self) -> np.ndarray:
        """View of the SLE-array stamps, shape (r', L')."""
        buf = (C.c_uint16 * self._n_slea).from_address(lib().or_slea_ptr(self._h))
        return np.frombuffer(buf, dtype=np.uint16).reshape(self.params["rp"], self.row_len)

    def hash(self, which: int, row: int, x: int) -> int:
        return int(lib().or_hash(self._h, which, row, x))

    # --- method -------------------------------------------------------------------------
    def ingest(self, pkts: np.ndarray, slice_: int) -> int:
        pkts = np.ascontiguousarray(pkts, dtype=np.uint32)
        return int(lib().or_ingest(self._h, _ptr(pkts), pkts.shape[0], slice_))

    def ingest_threads(self, pkts: np.ndarray, slice_: int, threads: int | None = None) -> int:
        """The same update with the rows split over threads (state identical to ingest)."""
        pkts = np.ascontiguousarray(pkts, dtype=np.uint32)
        return int(lib().or_ingest_threads(self._h, _ptr(pkts), pkts.shape[0], slice_,
                                           threads or default_threads()))

    def set_slice(self, slice_: int) -> int:
        return int(lib().or_set_slice(self._h, slice_))

    def merge(self, srcs) -> int:
        arr = (C.c_void_p * len(srcs))(*[s._h.value for s in srcs])
        return int(lib().or_merge(self._h, arr, len(srcs)))

    def rebase(self, offset: int) -> int:
        """Shift every stamp and the current slice down by offset (0 = never written)."""
        return int(lib().or_rebase(self._h, offset))

    def row_live(self, k: int) -> np.ndarray:
        out = np.zeros(self.params["rp"], dtype=np.uint64)
        lib().or_row_live(self._h, k, _ptr(out))
        return out

    def hot(self, k: int) -> np.ndarray:
        p = self.params
        out = np.zeros((p["r"], 1 << p["q"]), dtype=np.uint8)
        lib().or_hot(self._h, k, _ptr(out))
        return out

    def join_brute(self, hot: np.ndarray, cap: int = 1 << 22, threads: int | None = None):
        hot = np.ascontiguousarray(hot, dtype=np.uint8)
        out = np.zeros(cap, dtype=np.uint32)
        n = int(lib().or_join_brute(self._h, _ptr(hot), _ptr(out), cap,
                                    threads or default_threads()))
        if n < 0 or n > cap:
            raise RuntimeError(f"join_brute: {n}")
        return out[:n].copy()

    def join_tuples(self, hot: np.ndarray, cap: int = 1 << 22, tuple_cap: int = 1 << 24,
                    levels: bool = False):
        """Candidates of the tuple-growing search; with levels=True also the tuple count after
        every row (entry i for row i >= 1; entry 0 unused)."""
        hot = np.ascontiguousarray(hot, dtype=np.uint8)
        out = np.zeros(cap, dtype=np.uint32)
        lv = np.zeros(self.params["r"], dtype=np.uint64)
        n = int(lib().or_join_tuples(self._h, _ptr(hot), _ptr(out), cap, tuple_cap, _ptr(lv)))
        if n < 0 or n > cap:
            raise RuntimeError(f"join_tuples: {n}")
        return (out[:n].copy(), lv) if levels else out[:n].copy()

    def features(self, k: int, hosts) -> np.ndarray:
        hosts = np.ascontiguousarray(hosts, dtype=np.uint32)
        x = np.zeros((hosts.shape[0], k), dtype=np.uint32)
        rc = lib().or_features(self._h, k, _ptr(hosts), hosts.shape[0], _ptr(x))
        if rc:
            raise RuntimeError(f"features: {rc}")
        return x

    def estimate_one(self, U: int, row_live: np.ndarray, threshold: float):
        rl = np.ascontiguousarray(row_live, dtype=np.uint64)
        flags = C.c_uint32(0)
        est = lib().or_estimate_one(self._h, U, _ptr(rl), threshold, C.byref(flags))
        return float(est), int(flags.value)

    def estimate_filter(self, k: int, threshold: float, cands, cap: int = 1 << 20):
        cands = np.ascontiguousarray(cands, dtype=np.uint32)
        out = np.zeros(cap, dtype=RESULT_DTYPE)
        n = int(lib().or_estimate_filter(self._h, k, threshold, _ptr(cands), cands.shape[0],
                                         _ptr(out), cap))
        if n < 0 or n > cap:
            raise RuntimeError(f"estimate_filter: {n}")
        return out[:n].copy()

    def scan(self, k: int, threshold: float, cap: int = 1 << 20, threads: int | None = None):
        """Returns (results, candidates): results ascending by host, candidates ascending."""
        out = np.zeros(cap, dtype=RESULT_DTYPE)
        ccap = 1 << 22
        cands = np.zeros(ccap, dtype=np.uint32)
        ncand = C.c_uint64(0)
        n = int(lib().or_scan(self._h, k, threshold, _ptr(out), cap, _ptr(cands), ccap,
                              C.byref(ncand), threads or default_threads()))
        if n < 0 or n > cap:
            raise RuntimeError(f"scan: {n}")
        return out[:n].copy(), cands[:ncand.value].copy()
