import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (runs the HIP kernels)")
    config.addinivalue_line("markers", "slow: long-running")


@pytest.fixture(scope="session")
def lib_built():
    """libcredit.so must exist; builds it when absent (never silently skips)."""
    from paper_2609_01864_amd import credit

    if not os.path.exists(credit.LIB_PATH):
        from paper_2609_01864_amd import build

        build.build(verbose=False)
    return credit.lib()


@pytest.fixture(scope="session")
def gpu_handle(lib_built):
    import torch

    if not torch.cuda.is_available():
        pytest.fail("GPU test collected on a machine without a GPU")
    from paper_2609_01864_amd import credit

    h = credit.Handle(0, load_default_model=False)
    yield h
    h.close()
