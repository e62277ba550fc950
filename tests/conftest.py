import os
import sys
from fractions import Fraction

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

GOLDEN = os.path.join(ROOT, "tests", "golden")


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (runs through the HIP library)")
    config.addinivalue_line("markers", "slow: long CPU test")


def load_table1():
    """Table 1 of the paper as exact fractions: (a[6], b[6][5], c[6], cs[6])."""
    rows = []
    with open(os.path.join(GOLDEN, "rkck_table1.txt")) as fh:
        for line in fh:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            rows.append([Fraction(x) for x in line.split()[1:]])
    a = [r[0] for r in rows]
    b = [r[1:6] for r in rows]
    c = [r[6] for r in rows]
    cs = [r[7] for r in rows]
    return a, b, c, cs


def load_constants():
    out = {}
    with open(os.path.join(GOLDEN, "paper_constants.txt")) as fh:
        for line in fh:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            name, val = line.split()[:2]
            out[name] = float(Fraction(val)) if "/" in val else float(val)
    return out


@pytest.fixture(scope="session")
def orc():
    from oracle import oracle as O
    O.lib()
    return O


@pytest.fixture(scope="session")
def table1():
    return load_table1()


@pytest.fixture(scope="session")
def consts():
    return load_constants()
