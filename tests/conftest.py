import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (runs through the HIP C ABI)")


@pytest.fixture(scope="session", autouse=True)
def _built_host_libs():
    """Builds the host-side generator and oracle libraries if missing."""
    import graphgen
    import oracle
    graphgen.build(force=False)
    oracle.build(force=False)
    yield


@pytest.fixture(scope="session")
def gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2103_13577_amd as pkg
    pkg.lib()  # fails loudly if the HIP library is missing
    return torch.device("cuda:0")
