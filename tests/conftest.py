import os
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

GOLDEN = os.path.join(ROOT, "tests", "golden")


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (runs through the C-ABI library)")
    config.addinivalue_line("markers", "slow: CPU test that takes more than ~10 s")


def load_matrix(name):
    return np.loadtxt(os.path.join(GOLDEN, name), comments="#")


def paper_values():
    out = {}
    with open(os.path.join(GOLDEN, "paper_values.txt")) as fh:
        for line in fh:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            key, val, digits = line.split()[:3]
            out[key] = (float(val), int(digits))
    return out


@pytest.fixture(scope="session")
def oracle_lib():
    from oracle import build
    build.build(force=False)
    from oracle import sim
    return sim
