import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: oracle runs that take more than a few seconds")


def pytest_collection_modifyitems(config, items):
    # GPU tests run in file order after the CPU tests of the same file; nothing else reorders.
    return


@pytest.fixture(scope="session")
def has_gpu():
    try:
        import torch
        return bool(torch.cuda.is_available())
    except Exception:
        return False
