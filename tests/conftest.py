import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    # the library's on-disk autotune cache: a fresh file per test session
    import tempfile
    os.environ.setdefault("LENS_TUNE_CACHE",
                          os.path.join(tempfile.mkdtemp(prefix="lens_tune_"), "autotune.txt"))
    config.addinivalue_line("markers", "gpu: needs an MI355X (runs through the HIP library)")
    config.addinivalue_line("markers", "slow: long-running test")


def _gpu_available() -> bool:
    try:
        import torch
        return torch.cuda.is_available()
    except Exception:
        return False


def pytest_collection_modifyitems(config, items):
    if _gpu_available():
        return
    skip = pytest.mark.skip(reason="no GPU visible (run with -m gpu on an MI355X)")
    for it in items:
        if "gpu" in it.keywords:
            it.add_marker(skip)


@pytest.fixture(scope="session")
def lf():
    """The GPU package; fails loudly if the HIP library is not built."""
    import paper_2211_00354_amd as pkg
    pkg._lib.load()
    return pkg


@pytest.fixture(scope="session")
def dev():
    import torch
    return torch.device("cuda", 0)
