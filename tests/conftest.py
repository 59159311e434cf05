import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an AMD Instinct GPU (runs the HIP library)")


@pytest.fixture(scope="session")
def orc():
    import oracle

    oracle.build()
    return oracle


@pytest.fixture(scope="session")
def fv():
    """The HIP library binding; fails loudly when the library is not built."""
    import paper_1602_04386_amd as fvmod

    fvmod.lib()
    return fvmod


@pytest.fixture(scope="session")
def ctx(fv):
    c = fv.Context(0)
    yield c
    c.close()
