import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")


def read_golden(name):
    """Parse a tests/golden fixture: header line 'f_min f_max nd', then Nf input
    rows, then nd expected rows (integers)."""
    import numpy as np
    path = os.path.join(ROOT, "tests", "golden", name)
    rows = [l.split() for l in open(path) if l.strip() and not l.lstrip().startswith("#")]
    f_min, f_max, nd = float(rows[0][0]), float(rows[0][1]), int(rows[0][2])
    data = np.array([[int(v) for v in r] for r in rows[1:]], dtype=np.int64)
    nf = len(data) - nd
    return f_min, f_max, nd, data[:nf], data[nf:]


@pytest.fixture(scope="session")
def gpu_available():
    import torch
    return torch.cuda.is_available()
