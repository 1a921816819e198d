import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (runs through the HIP library)")
    config.addinivalue_line("markers", "slow: larger cases (full benchmark sizes on the GPU, larger CPU cases)")


@pytest.fixture(scope="session")
def ora():
    from oracle import oracle as O
    if not os.path.exists(O.LIB):
        O.build()
    return O
