import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

GOLDEN = os.path.join(ROOT, "tests", "golden")


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU")
    config.addinivalue_line("markers", "slow: long-running CPU test")


def read_table(name):
    """Two-column integer fixture under tests/golden (comments start with #)."""
    out = {}
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            k, v = line.split()
            out[int(k)] = int(v)
    return out


@pytest.fixture(scope="session")
def paper_pow10():
    return read_table("paper_pi_pow10.txt")


@pytest.fixture(scope="session")
def paper_pow2():
    return read_table("paper_pi_pow2.txt")


@pytest.fixture(scope="session")
def pc():
    """The HIP library's Python binding (raises if libpicount.so is missing)."""
    import paper_1503_01839_amd as pc
    pc.lib()
    return pc
