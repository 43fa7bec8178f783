import os
import sys

import pytest

REPO = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if REPO not in sys.path:
    sys.path.insert(0, REPO)

GOLDEN = os.path.join(REPO, "tests", "golden")


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: long CPU test, excluded from the default quick run")


def load_table1():
    """Table 1 of the paper as {n: dict} (see tests/golden/table1.txt)."""
    rows = {}
    with open(os.path.join(GOLDEN, "table1.txt")) as fh:
        for line in fh:
            line = line.split("#", 1)[0].split()
            if not line:
                continue
            v = [None if t == "-" else float(t) for t in line]
            n = int(v[0])
            rows[n] = {
                "fp64": {"N": int(v[1]), "eb0": v[2], "ebn1": v[3], "ebn": v[4], "en": v[5]},
                "fp32": {"N": int(v[6]), "eb0": v[7], "ebn1": v[8], "ebn": v[9], "en": v[10]},
            }
    return rows


@pytest.fixture(scope="session")
def table1():
    return load_table1()
