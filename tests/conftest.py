import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: longer CPU test")


def load_golden(name):
    """Parse a tests/golden/*.txt fixture into {section: [[numbers...]]}."""
    path = os.path.join(ROOT, "tests", "golden", name)
    out, cur = {}, None
    with open(path) as fh:
        for line in fh:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            if line[0].isalpha():
                cur = line
                out[cur] = []
            else:
                out[cur].append([float(x) for x in line.split()])
    return out
