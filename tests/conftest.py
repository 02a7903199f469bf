import json
import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

GOLDEN = os.path.join(ROOT, "tests", "golden")


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU")
    config.addinivalue_line("markers", "slow: takes tens of seconds on the CPU")


def golden(name):
    with open(os.path.join(GOLDEN, name)) as f:
        return json.load(f)


@pytest.fixture(scope="session")
def c1_stream():
    from synth import make_stream
    from synth.configs import C1_RECIPE
    return make_stream(C1_RECIPE)


@pytest.fixture(scope="session")
def c1_oracle(c1_stream):
    """Oracle sketch fed the whole config-1 stream, plus per-slice snapshots of its scans."""
    import oracle
    from synth.configs import C1_PARAMS
    sk = oracle.OracleSketch(C1_PARAMS)
    for s in range(1, c1_stream.recipe.n_slices + 1):
        assert sk.ingest(c1_stream.slice_pkts(s), s) == 0
    return sk
