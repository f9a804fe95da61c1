import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: larger CPU cases")


_CASES = {}


def cached_case(name, **over):
    """Build (once per session) a named workload, optionally with spec overrides."""
    from paper_2002_05019_amd.problem import make_case, named_spec
    key = (name, tuple(sorted(over.items())))
    if key not in _CASES:
        spec = named_spec(name)
        for k, v in over.items():
            setattr(spec, k, v)
        _CASES[key] = make_case(spec)
    return _CASES[key]


@pytest.fixture(scope="session")
def case_cache():
    return cached_case
