import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (runs the HIP library)")
    config.addinivalue_line("markers", "slow: full-size workload (minutes on the CPU)")


@pytest.fixture(scope="session")
def gpu():
    """The loaded GPU library; fails (does not skip) when the HIP extension is
    missing on a machine that has a GPU."""
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU in this container")
    from paper_1504_05022_amd import lib
    return lib.load()
