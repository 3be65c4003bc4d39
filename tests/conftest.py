import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: longer CPU-only checks")


_CACHE = {}


def cached(key, fn):
    if key not in _CACHE:
        _CACHE[key] = fn()
    return _CACHE[key]


@pytest.fixture(scope="session")
def cube4():
    from harness import unit_cube_problem
    return cached("cube4", lambda: unit_cube_problem())


@pytest.fixture(scope="session")
def cube4_h(cube4):
    import oracle
    return cached("cube4_h", lambda: oracle.setup(cube4))
