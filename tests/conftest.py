import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU")
    config.addinivalue_line("markers", "slow: long CPU run, excluded from the default CPU suite")


def load_matrix(name):
    """Read a golden matrix fixture (rows of integers or fractions, '#' comments)."""
    from fractions import Fraction

    import numpy as np

    path = os.path.join(ROOT, "tests", "golden", name)
    rows = [line.split() for line in open(path) if line.strip() and not line.startswith("#")]
    return np.array([[float(Fraction(x)) for x in r] for r in rows])


@pytest.fixture(scope="session")
def oracle_mod():
    import oracle

    oracle.build(force=False)
    return oracle
