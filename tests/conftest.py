import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (runs through the HIP C-ABI library)")
    config.addinivalue_line("markers", "slow: long oracle physics runs (still part of the CPU suite)")


@pytest.fixture(scope="session", autouse=True)
def _threads():
    import torch
    torch.set_num_threads(min(8, os.cpu_count() or 1))
    yield
