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
    config.addinivalue_line("markers", "slow: full-size case (seconds to minutes)")


def load_golden(name):
    """Parse a `key: v v v` fixture; repeated keys become lists of rows."""
    out = {}
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            key, rest = line.split(":", 1)
            vals = [float(t) for t in rest.split()]
            out.setdefault(key.strip(), []).append(vals)
    return out


@pytest.fixture
def example():
    """The Example matrix of Fig. 1 as CSR arrays built from its dense rows."""
    rows = np.array(load_golden("example_matrix.txt")["row"], dtype=np.float64)
    n = rows.shape[0]
    r, c = np.nonzero(rows)
    rowptr = np.zeros(n + 1, np.int32)
    np.cumsum(np.bincount(r, minlength=n), out=rowptr[1:])
    return dict(A=rows, n=n, rowptr=rowptr, colind=c.astype(np.int32), val=rows[r, c])
