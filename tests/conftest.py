import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (HIP device) and libtrstream.so")
    config.addinivalue_line("markers", "slow: long-running CPU test")


@pytest.fixture(scope="session")
def trlib():
    """The built HIP library on a machine with a HIP device.  Fails loudly
    when the library is missing; skips only when there is no device."""
    import torch
    import paper_2307_00719_amd as P
    P.load()
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    return P
