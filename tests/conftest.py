import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
for p in (ROOT, os.path.join(ROOT, "tests")):
    if p not in sys.path:
        sys.path.insert(0, p)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (HIP device)")
    config.addinivalue_line("markers", "slow: longer CPU test")


def _ensure_built():
    from paper_2606_06135_amd.binding import LIB_PATH
    if not os.path.exists(LIB_PATH):
        from paper_2606_06135_amd import build
        build.build(verbose=False)


@pytest.fixture(scope="session")
def gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    _ensure_built()
    return torch.device("cuda:0")


@pytest.fixture(scope="session")
def hiplib():
    _ensure_built()
    from paper_2606_06135_amd import lib
    return lib()
