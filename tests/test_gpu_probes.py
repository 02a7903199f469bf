"""Measurement probes on the GPU: the replay probe's recorded cell list is exactly the set of
recorders an ingest writes, so replaying it with the ingest's stamp leaves the same state."""
import numpy as np
import pytest

from gpu_util import dev_pkts
from paper_1805_09246_amd import sps
from synth import make_stream
from synth.configs import C1_PARAMS, C1_RECIPE, C2_PARAMS, C2_SMALL_RECIPE

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("which", ["c1", "c2_shape"])
def test_replay_probe_writes_exactly_the_ingest_cells(which):
    rec, params = (C1_RECIPE, C1_PARAMS) if which == "c1" else (C2_SMALL_RECIPE, C2_PARAMS)
    st = make_stream(rec)
    a, b = sps.Sketch(params), sps.Sketch(params)
    for s in (1, 2, 3):
        p = dev_pkts(st.slice_pkts(s))
        print(f"replay probe {which}: slice {s}, {p.shape[0]} pairs", flush=True)
        a.ingest(p, s)
        cells, off = sps.sps_probe_replay_record(b.h, p)
        n = p.shape[0]
        total = off[8]
        assert all(off[c] <= off[c + 1] for c in range(8))
        assert total >= params["rp"] * n and (total - params["rp"] * n) % params["r"] == 0
        sps.sps_probe_replay(b.h, cells, off, s)
    sa, la = a.state()
    sb, lb = b.state()
    assert np.array_equal(sa, sb)
    assert np.array_equal(la, lb)
    a.close()
    b.close()
