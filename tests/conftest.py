import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)
HERE = os.path.dirname(os.path.abspath(__file__))
if HERE not in sys.path:
    sys.path.insert(0, HERE)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs a real MI355X (gfx950) GPU and the built HIP library")


@pytest.fixture
def golden():
    """Load a ``key value`` fixture from tests/golden/ (lines starting with # are comments)."""
    def load(name):
        out = {}
        with open(os.path.join(HERE, "golden", name)) as f:
            for line in f:
                line = line.strip()
                if not line or line.startswith("#"):
                    continue
                k, v = line.split()[:2]
                out[k] = float(v)
        return out
    return load
