import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU")
    config.addinivalue_line("markers", "slow: longer CPU checks")


@pytest.fixture(scope="session")
def ico():
    """Cached icosphere meshes by level."""
    from synthetic import icosphere
    cache = {}

    def get(level):
        if level not in cache:
            cache[level] = icosphere(level)
        return cache[level]
    return get


@pytest.fixture(scope="session")
def oracle_ops(ico):
    """Cached oracle operators (and dense matrices for small levels)."""
    from oracle import bem
    cache = {}

    def get(level, dense=False):
        if level not in cache:
            V, T = ico(level)
            cache[level] = [bem.Operator(V, T), None]
        if dense and cache[level][1] is None:
            cache[level][1] = cache[level][0].dense()
        return cache[level][0], cache[level][1]
    return get
