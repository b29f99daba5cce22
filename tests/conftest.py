import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")


@pytest.fixture(scope="session")
def orc():
    from oracle import oracle

    oracle.lib()  # builds liboracle.so with gcc if it is missing or stale
    return oracle


@pytest.fixture(scope="session")
def gpu():
    """The binding module, on a machine with a GPU; fails loudly if the library is missing."""
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1312_2234_amd import lbm

    lbm.lib()
    return lbm
