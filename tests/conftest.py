import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU")
    config.addinivalue_line("markers", "slow: long-running CPU test")


@pytest.fixture(scope="session")
def orc():
    import oracle
    oracle.build(force=False)
    return oracle


@pytest.fixture(scope="session")
def ag():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    import paper_2010_13792_amd as ag
    ag.load_library()
    return ag


@pytest.fixture(scope="module")
def ctx(ag):
    c = ag.Context(0)
    yield c
    c.close()


def rel_err(a, b):
    """Per-row |a - b| / |b| (vector or tensor rows)."""
    import numpy as np
    a = np.asarray(a).reshape(len(a), -1)
    b = np.asarray(b).reshape(len(b), -1)
    return np.linalg.norm(a - b, axis=1) / np.linalg.norm(b, axis=1)


def tensor_rel_err(t, tref):
    """Frobenius-relative error of (n, 6) symmetric tensors (off-diagonals twice)."""
    import numpy as np
    w = np.array([1, 1, 1, 2, 2, 2], dtype=float)
    d = np.sqrt(((np.asarray(t) - tref) ** 2 * w).sum(1))
    return d / np.sqrt((np.asarray(tref) ** 2 * w).sum(1))
