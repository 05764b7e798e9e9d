import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU")
    config.addinivalue_line("markers", "slow: long-running case")


def load_golden(name):
    """Parse a tests/golden fixture into (n, source, edges, expected)."""
    path = os.path.join(ROOT, "tests", "golden", name)
    n = src = None
    edges, expect = [], {}
    with open(path) as f:
        for line in f:
            line = line.split("#", 1)[0].strip()
            if not line:
                continue
            tok = line.split()
            if tok[0] == "n":
                n = int(tok[1])
            elif tok[0] == "source":
                src = int(tok[1])
            elif tok[0] == "edge":
                edges.append((int(tok[1]), int(tok[2]), int(tok[3])))
            elif tok[0] == "expect":
                expect[int(tok[1])] = int(tok[2])
    return n, src, edges, expect


@pytest.fixture(scope="session")
def golden():
    return load_golden
