import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU")
    config.addinivalue_line("markers", "slow: takes more than a few seconds on CPU")


@pytest.fixture(scope="session")
def gpu_lib():
    """The built HIP library, loaded through its Python binding.

    GPU tests need both the library and a visible device; a missing library on
    a GPU host is an error, not a skip.
    """
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU visible")
    from paper_1003_3272_amd import nmf
    return nmf.load()
