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
    config.addinivalue_line("markers", "slow: takes more than a few seconds on the CPU")


def read_golden(name: str) -> dict:
    """Parse a golden fixture: '#' comments, a key line, then rows of numbers."""
    out, key, rows = {}, None, []
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            try:
                vals = [float(t) for t in line.split()]
            except ValueError:
                if key is not None:
                    out[key] = np.array(rows if len(rows) > 1 else rows[0])
                key, rows = line, []
                continue
            rows.append(vals)
    if key is not None:
        out[key] = np.array(rows if len(rows) > 1 else rows[0])
    return out


@pytest.fixture(scope="session")
def golden_csr_example():
    return read_golden("csr_example.txt")
