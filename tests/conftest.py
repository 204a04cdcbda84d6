import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: longer CPU test")


_CACHE = {}


@pytest.fixture(scope="session")
def crystal_cache():
    """Session cache of seeded crystals keyed by (name, kwargs)."""
    from synth import crystal_for

    def get(name, **kw):
        key = (name, tuple(sorted((k, repr(v)) for k, v in kw.items())))
        if key not in _CACHE:
            _CACHE[key] = crystal_for(name, **kw)
        return _CACHE[key]
    return get
