import os
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

GOLDEN = os.path.join(ROOT, "tests", "golden")


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: long-running GPU parity case at full workload size")


def load_inputs(config: int):
    """Stored workload inputs written by tests/golden/make_inputs.py."""
    import synthlens as S
    d = np.load(os.path.join(GOLDEN, f"config{config}_inputs.npz"))
    x0, y0, h, nx, ny = d["grid"]
    grid = S.Grid(float(x0), float(y0), float(h), int(nx), int(ny))
    obs = dict(sys_off=d["sys_off"].astype(np.int32), x=d["x"], y=d["y"], sigma=d["sigma"], dls=d["dls"])
    return d["params"], grid, obs


@pytest.fixture(scope="session")
def inputs():
    return load_inputs
