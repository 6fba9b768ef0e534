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
    config.addinivalue_line("markers", "slow: long-running CPU test")


def read_golden(name):
    """Non-comment lines of a golden fixture, split into sections at comment lines."""
    sections, cur = [], []
    with open(os.path.join(GOLDEN, name)) as fh:
        for line in fh:
            s = line.strip()
            if not s:
                continue
            if s.startswith("#"):
                if cur:
                    sections.append(cur)
                    cur = []
                continue
            cur.append(s.split())
    if cur:
        sections.append(cur)
    return sections


@pytest.fixture
def rng():
    return np.random.default_rng(12345)
