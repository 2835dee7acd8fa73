import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

# PyTorch ships its own HIP runtime.  Importing it before the library is loaded (as bench.py
# does) lets the library and PyTorch share one runtime, so the tests of the PyTorch stream and
# allocator interop see the device.  Importing touches no device.
import torch  # noqa: E402,F401


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (HIP device)")
    config.addinivalue_line("markers", "slow: long-running CPU test")


@pytest.fixture(scope="session")
def oracle_mod():
    import oracle
    oracle._load()
    return oracle


@pytest.fixture(scope="session")
def perm(oracle_mod):
    """perm[k] = library index of the oracle's velocity k."""
    from _helpers import perm_lib_to_oracle
    return perm_lib_to_oracle(oracle_mod)
