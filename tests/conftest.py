import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU")
    config.addinivalue_line("markers", "slow: CPU test that runs the oracle for tens of seconds")


def gpu_available():
    try:
        import torch
        return torch.cuda.is_available()
    except Exception:
        return False


@pytest.fixture(scope="session")
def P():
    """The product binding.  Builds the library once if nothing is built yet;
    GPU tests fail loudly if it cannot load."""
    lib = os.path.join(ROOT, "paper_2312_00369_amd", "libpflbm.so")
    if not os.path.exists(lib):
        from paper_2312_00369_amd.build import build
        build(verbose=False)
    import paper_2312_00369_amd as P
    return P
