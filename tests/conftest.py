import os
import sys
from pathlib import Path

import pytest

ROOT = Path(__file__).resolve().parent.parent
sys.path.insert(0, str(ROOT))
sys.path.insert(0, str(Path(__file__).resolve().parent))


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: large CPU work (full-size workload generation)")


_CACHE = {}


def cached(name, fn):
    if name not in _CACHE:
        _CACHE[name] = fn()
    return _CACHE[name]


@pytest.fixture(scope="session")
def small_workload():
    from synth import configs
    return cached("small", configs.small)


@pytest.fixture(scope="session")
def medium_workload():
    from synth import configs
    return cached("medium", configs.medium)


@pytest.fixture(scope="session")
def large_workload():
    from synth import configs
    return cached("large", configs.large)


@pytest.fixture(scope="session")
def wide_workload():
    from synth import configs
    return cached("wide", configs.wide)
