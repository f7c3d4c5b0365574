import pathlib
import sys

import pytest

ROOT = pathlib.Path(__file__).resolve().parent.parent
if str(ROOT) not in sys.path:
    sys.path.insert(0, str(ROOT))


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs a HIP device (runs the liblbm kernels)")
    config.addinivalue_line("markers", "slow: long CPU run, excluded from the quick suite")


@pytest.fixture(scope="session")
def gpu():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no HIP device visible")
    import paper_2002_05265_amd.binding as B

    B.lib()  # fails loudly if the HIP library is missing
    return torch.device("cuda:0")
