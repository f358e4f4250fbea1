import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs a HIP device (MI355X); parity of the HIP path against the oracle")
    config.addinivalue_line("markers", "slow: takes more than a few seconds")


@pytest.fixture(scope="session")
def orc():
    import oracle
    oracle.build(force=False)
    return oracle


@pytest.fixture(scope="session")
def mbe():
    """The HIP library binding; fails loudly when the library or the device is missing."""
    import torch
    if not torch.cuda.is_available():
        pytest.fail("GPU test run without a HIP device")
    import paper_2401_05039_amd as m
    m.load()
    return m
