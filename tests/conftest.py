import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")


def golden(name):
    path = os.path.join(ROOT, "tests", "golden", "paper_values.txt")
    for line in open(path):
        line = line.strip()
        if not line or line.startswith("#"):
            continue
        k, v, _cite = line.split()
        if k == name:
            return float(v)
    raise KeyError(name)


@pytest.fixture
def paper():
    return golden
