import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built device library")
    config.addinivalue_line("markers", "slow: takes more than a few seconds on the CPU")


_GRIDS = {}


@pytest.fixture(scope="session")
def grids():
    """Session cache of generated grids, keyed by spec name."""
    import gridgen

    class _Cache:
        def __getitem__(self, key):
            if key not in _GRIDS:
                _GRIDS[key] = gridgen.make_grid(key)
            return _GRIDS[key]

    return _Cache()
