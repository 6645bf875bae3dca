import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (runs through the HIP C ABI)")
    config.addinivalue_line("markers", "slow: larger CPU cases")


@pytest.fixture(scope="session")
def oracle():
    from oracle import ref
    ref.load()
    return ref


def read_golden(name):
    """Parse a tests/golden/*.txt fixture into {section: numpy array}."""
    import numpy as np
    out, cur, rows = {}, None, []
    with open(os.path.join(ROOT, "tests", "golden", name)) as f:
        for line in f:
            line = line.split("#", 1)[0].strip()
            if not line:
                continue
            if line.startswith("["):
                if cur is not None:
                    out[cur] = np.array(rows, dtype=float)
                cur, rows = line.strip("[]"), []
            else:
                rows.append([float(t) for t in line.split()])
    if cur is not None:
        out[cur] = np.array(rows, dtype=float)
    return out
