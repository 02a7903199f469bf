"""Helpers shared by the GPU parity tests: move packets to the device, compare a GPU sketch
with the oracle (state, scan stages, results)."""
import numpy as np
import torch

from paper_1805_09246_amd import sps

ULP_TOL = 4


def dev_pkts(p: np.ndarray) -> torch.Tensor:
    p = np.ascontiguousarray(p, dtype=np.uint32)
    return torch.from_numpy(p.view(np.int32)).to("cuda")


def assert_state_equal(g: "sps.Sketch", o, where=""):
    sre, slea = g.state()
    assert sre.shape == o.sre().shape and slea.shape == o.slea().shape
    if not np.array_equal(sre, o.sre()):
        bad = np.argwhere(sre != o.sre())
        raise AssertionError(f"{where}: SRE differs at {len(bad)} cells, first {bad[:3].tolist()}")
    if not np.array_equal(slea, o.slea()):
        bad = np.argwhere(slea != o.slea())
        raise AssertionError(f"{where}: SLE array differs at {len(bad)} cells, first {bad[:3].tolist()}")
    assert g.cur == o.cur, where


def gpu_hot(g: "sps.Sketch") -> np.ndarray:
    p = g.params
    buf = sps.sps_debug_copy(g.h, 0)
    bits = np.unpackbits(buf, bitorder="little")
    return bits.reshape(p["r"], 1 << p["q"]).astype(np.uint8)


def gpu_candidates(g: "sps.Sketch") -> np.ndarray:
    return np.sort(sps.sps_debug_copy(g.h, 1).view(np.uint32))


def gpu_row_live(g: "sps.Sketch") -> np.ndarray:
    return sps.sps_debug_copy(g.h, 2).view(np.uint32).astype(np.uint64)


def assert_estimates_close(a, b, where=""):
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    tol = ULP_TOL * np.spacing(np.maximum(np.abs(a), np.abs(b)))
    bad = np.abs(a - b) > tol
    assert not bad.any(), f"{where}: estimates differ beyond {ULP_TOL} ulp: {a[bad][:3]} vs {b[bad][:3]}"


def assert_scan_equal(g: "sps.Sketch", o, k: int, threshold: float, where=""):
    got = g.scan(k, threshold, cap=1 << 18)
    # stage 1: row live counts and hot SREs
    assert np.array_equal(gpu_row_live(g), o.row_live(k)), f"{where}: row live counts"
    ohot = o.hot(k)
    assert np.array_equal(gpu_hot(g), ohot), f"{where}: hot SREs"
    want, ocand = o.scan(k, threshold)
    # stage 2: candidates (unique; order checked on the final list)
    assert np.array_equal(gpu_candidates(g), ocand), f"{where}: candidates"
    # stages 3-4: estimates, filter, order
    near = (want["flags"] & sps.F_NEAR) != 0
    assert not near.any(), f"{where}: a candidate lies within 1e-9 of the threshold"
    assert np.array_equal(got["host"], want["host"]), f"{where}: reported hosts"
    assert np.array_equal(got["live"], want["live"]), f"{where}: |USLE|^k"
    assert np.array_equal(got["flags"], want["flags"]), f"{where}: flags"
    assert_estimates_close(got["estimate"], want["estimate"], where)
    return got


def import_state(g: "sps.Sketch", sre: np.ndarray, slea: np.ndarray, cur: int):
    """Give a GPU sketch exactly this state (u16 stamps, shapes as in Sketch.state()) through
    the checkpoint entry points."""
    if g.cur < cur:
        g.advance(cur)
    buf = g.export()
    body = buf[sps.HEADER_BYTES:].view(np.uint16)
    body[: sre.size] = sre.ravel()
    body[sre.size: sre.size + slea.size] = slea.ravel()
    g.import_(buf)
    assert g.cur == cur


def assert_results_equal(got, want, where=""):
    """Full result records: hosts, |USLE|^k and flags exact, estimates within ULP_TOL ulp."""
    assert len(got) == len(want), f"{where}: {len(got)} results, oracle {len(want)}"
    assert np.array_equal(got["host"], want["host"]), f"{where}: hosts"
    assert np.array_equal(got["live"], want["live"]), f"{where}: |USLE|^k"
    assert np.array_equal(got["flags"], want["flags"]), f"{where}: flags"
    assert_estimates_close(got["estimate"], want["estimate"], where)
