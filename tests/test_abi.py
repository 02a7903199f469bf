"""The C-ABI library loads and exports every symbol include/sps.h declares; host-only entry
points (parameter validation, sizes, error strings) work without a GPU."""
import json
import os
import re

import pytest

from conftest import ROOT


def _declared():
    text = open(os.path.join(ROOT, "include", "sps.h")).read()
    return sorted(set(re.findall(r"^(?:int|const char\*)\s+(sps_\w+)\s*\(", text, re.M)))


@pytest.fixture(scope="module")
def L():
    from paper_1805_09246_amd import sps
    if not os.path.exists(sps.LIB_PATH):
        import __graft_entry__
        __graft_entry__.build()
    return sps


def test_exports_every_declared_symbol(L):
    names = _declared()
    assert len(names) >= 20
    lib = L.lib()
    for n in names:
        assert hasattr(lib, n), n
    assert sorted(L.EXPORTS) == names


def test_no_cpu_fallback_in_binding():
    src = open(os.path.join(ROOT, "paper_1805_09246_amd", "sps.py")).read()
    assert "import oracle" not in src and "from oracle" not in src
    for f in os.listdir(os.path.join(ROOT, "paper_1805_09246_amd", "csrc")):
        assert "oracle" not in open(os.path.join(ROOT, "paper_1805_09246_amd", "csrc", f)).read()


def test_sketch_bytes_and_validation(L):
    from synth.configs import C1_PARAMS, C2_PARAMS
    n1 = L.sps_sketch_bytes(C1_PARAMS)
    # SRE 6*4096*8*2 + SLE 5*4096*1024*2 + workspace
    assert n1 > 6 * 4096 * 16 + 5 * 4096 * 1024 * 2
    assert L.sps_sketch_bytes(C2_PARAMS) > 640 * 2 ** 20
    bad = [
        dict(C1_PARAMS, r=5),            # (r-2)*delta + q = 27 < 32
        dict(C1_PARAMS, eta=6),
        dict(C1_PARAMS, etap=1000),
        dict(C1_PARAMS, deltap=2048),    # delta' > eta'
        dict(C1_PARAMS, rp=9),
        dict(C1_PARAMS, q=5),
        dict(C1_PARAMS, theta=0),
        dict(C1_PARAMS, anet_side=2),
        dict(C1_PARAMS, delta=12),       # delta >= q
    ]
    for p in bad:
        with pytest.raises(L.SpsError) as e:
            L.sps_sketch_bytes(p)
        assert e.value.code == L.SPS_EINVAL
    assert L.sps_sketch_bytes(dict(C1_PARAMS, deltap=16)) < n1


def test_strerror(L):
    for code in range(0, -8, -1):
        assert len(L.strerror(code)) >= 2
    assert L.strerror(-99) == "unknown error"


def test_binding_constants_match_header():
    """Every numeric #define of include/sps.h that the binding mirrors has the same value."""
    from paper_1805_09246_amd import sps
    text = open(os.path.join(ROOT, "include", "sps.h")).read()
    defs = {m.group(1): int(m.group(2)) for m in
            re.finditer(r"^#define SPS_(\w+) \(?(-?\d+)u?\)?", text, re.M)}
    pairs = {f"SPS_{k}": v for k, v in defs.items() if k.startswith("E") or k == "OK"}
    pairs.update({k: v for k, v in defs.items() if k.startswith(("F_", "INFO_", "MODE_"))})
    pairs.update({k: v for k, v in defs.items() if k in ("MLP_IN", "MLP_HIDDEN")})
    checked = 0
    for name, v in pairs.items():
        assert hasattr(sps, name), name
        assert getattr(sps, name) == v, name
        checked += 1
    assert checked >= 20
    stages = {k[len("STAGE_"):].lower(): v for k, v in defs.items() if k.startswith("STAGE_")}
    assert stages == {n: j for j, n in enumerate(sps.STAGES)}
    assert defs["NSTAGES"] == len(sps.STAGES)


def test_packet_batches_rejected_before_launch():
    """Every ingest binding refuses a packet tensor that is not (n, 2) x 32 bits on the device
    before it touches the library: a flat (2n,) tensor would otherwise be read as 2n pairs."""
    import ctypes as C

    import torch

    from paper_1805_09246_amd import sps
    h = C.c_void_p(1)  # never dereferenced: the check comes first
    flat = torch.zeros(20, dtype=torch.int32)
    wide = torch.zeros((10, 2), dtype=torch.int64)
    host = torch.zeros((10, 2), dtype=torch.int32)  # right shape, but not device memory
    for bad in (flat, wide, host):
        with pytest.raises(ValueError):
            sps.sps_ingest(h, bad, 1)
        with pytest.raises(ValueError):
            sps.sps_ingest_batched([h, h], [torch.zeros((0, 2), dtype=torch.int32), bad], 1)
        with pytest.raises(ValueError):
            sps.sps_autotune_ingest([h], [bad], 1)
    with pytest.raises(ValueError):
        sps.sps_ingest_batched([h], [host, host], 1)  # one sketch, two batches


def test_tuning_cache_file_round_trip(tmp_path):
    """The tuning cache reads back what it writes, keys entries by architecture, shape and
    batched flag, replaces equal keys on load, and refuses malformed files whole."""
    from paper_1805_09246_amd import sps
    shape = dict(q=14, r=11, delta=2, eta=8, qp=16, rp=5, etap=1024, deltap=1024, theta=1024,
                 anet_side=0, seed=1)
    sps.sps_tuning_cache_clear()
    assert sps.sps_tuning_lookup(shape, False, arch="gfx950") is None
    f = tmp_path / "tune.json"
    f.write_text(
        '{"sps_tuning_cache": 1, "entries": [\n'
        '{"arch": "gfx950", "q": 14, "r": 11, "delta": 2, "eta": 8, "qp": 16, "rp": 5, '
        '"etap": 1024, "deltap": 1024, "mode": 0, "batched": 0, "blocks_per_cu": 32, '
        '"batch_tile": 4096, "host_classes": 8},\n'
        '{"arch": "gfx950", "q": 14, "r": 11, "delta": 2, "eta": 8, "qp": 16, "rp": 5, '
        '"etap": 1024, "deltap": 1024, "mode": 0, "batched": 1, "blocks_per_cu": 8, '
        '"batch_tile": 2048, "host_classes": 1}\n]}\n')
    sps.sps_tuning_cache_load(str(f))
    one = sps.sps_tuning_lookup(shape, False, arch="gfx950")
    assert one == {"blocks_per_cu": 32, "batch_tile": 4096, "host_classes": 8}
    assert sps.sps_tuning_lookup(shape, True, arch="gfx950") == \
        {"blocks_per_cu": 8, "batch_tile": 2048, "host_classes": 1}
    assert sps.sps_tuning_lookup(shape, False, arch="gfx942") is None
    assert sps.sps_tuning_lookup(dict(shape, qp=15), False, arch="gfx950") is None
    out = tmp_path / "out.json"
    sps.sps_tuning_cache_save(str(out))
    json.loads(out.read_text())  # valid JSON
    sps.sps_tuning_cache_clear()
    sps.sps_tuning_cache_load(str(out))
    assert sps.sps_tuning_lookup(shape, False, arch="gfx950") == one
    # a file with a bad entry adds nothing
    bad = tmp_path / "bad.json"
    bad.write_text(f.read_text().replace('"host_classes": 1', '"host_classes": 3'))
    sps.sps_tuning_cache_clear()
    with pytest.raises(sps.SpsError):
        sps.sps_tuning_cache_load(str(bad))
    assert sps.sps_tuning_lookup(shape, False, arch="gfx950") is None
    with pytest.raises(sps.SpsError):
        sps.sps_tuning_cache_load(str(tmp_path / "missing.json"))
    sps.sps_tuning_cache_clear()
