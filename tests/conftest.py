import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (runs through the HIP library)")
    config.addinivalue_line("markers", "slow: larger CPU cases")


@pytest.fixture(scope="session")
def gen():
    import fsigen
    return fsigen


_cache = {}


def system(name, seed=0, t_phase=0.0):
    """Session cache of generated systems (they are read-only)."""
    import fsigen
    key = (name, seed, t_phase)
    if key not in _cache:
        _cache[key] = fsigen.generate(name, seed=seed, t_phase=t_phase)
    return _cache[key]
