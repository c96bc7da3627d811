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


def read_golden(name):
    """Parse a golden text fixture: '#' comments, named sections of integer rows."""
    sections, cur = {}, None
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            if line[0].isalpha():
                cur = line
                sections[cur] = []
                continue
            sections.setdefault(cur, []).append([int(x) for x in line.split()])
    return {k: np.array(v) for k, v in sections.items()}


@pytest.fixture(scope="session")
def oracle_lib():
    import oracle

    oracle._load()
    return oracle
