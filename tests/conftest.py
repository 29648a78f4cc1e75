import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")


@pytest.fixture(scope="session", autouse=True)
def _cpu_helpers_built():
    # The generator and the oracle are small C/C++ libraries; build them if a
    # fresh checkout has no binaries yet (a no-op when they are up to date).
    import gen
    import oracle
    gen.build()
    oracle.build()
    yield


@pytest.fixture(scope="session")
def gpu():
    """The product binding, loaded on cuda:0; skips the test when no GPU is visible."""
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU visible")
    from paper_2512_02862_amd import pyst
    pyst.load()
    return pyst
