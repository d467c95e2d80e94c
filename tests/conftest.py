import os
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (runs through the HIP library)")
    config.addinivalue_line("markers", "slow: larger CPU-only oracle checks")


def read_golden(name):
    """Parse a tests/golden block file: 'name rows cols' headers followed by rows."""
    path = os.path.join(ROOT, "tests", "golden", name)
    blocks, lines = {}, []
    with open(path) as fh:
        for ln in fh:
            ln = ln.strip()
            if ln and not ln.startswith("#"):
                lines.append(ln)
    i = 0
    while i < len(lines):
        key, r, c = lines[i].split()
        r, c = int(r), int(c)
        rows = [list(map(float, lines[i + 1 + q].split())) for q in range(r)]
        A = np.array(rows, dtype=float)
        assert A.shape == (r, c), (key, A.shape)
        blocks[key] = A
        i += 1 + r
    return blocks


@pytest.fixture
def golden():
    return read_golden
