import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: long CPU test")


def read_golden(name):
    """Read a whitespace matrix fixture; returns (matrix, factor)."""
    import numpy as np
    factor = 1.0
    rows = []
    with open(os.path.join(ROOT, "tests", "golden", name)) as fh:
        for line in fh:
            line = line.strip()
            if not line:
                continue
            if line.startswith("#"):
                if line.startswith("# factor"):
                    num, den = line.split()[2].split("/")
                    factor = float(num) / float(den)
                continue
            rows.append([float(v) for v in line.split()])
    return np.array(rows), factor
