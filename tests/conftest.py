import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) and the built HIP library")
    config.addinivalue_line("markers", "slow: longer CPU test")


@pytest.fixture(scope="session")
def rng():
    import numpy as np

    return np.random.default_rng(12345)


def _ensure_lib():
    from paper_2006_11851_amd import pts

    if not os.path.exists(pts.LIB_PATH):
        from paper_2006_11851_amd import build

        build.build()
    return pts


@pytest.fixture(scope="session")
def ptslib():
    return _ensure_lib()


@pytest.fixture(scope="session")
def gpu_ctx():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    pts = _ensure_lib()
    return pts.Context(0)
