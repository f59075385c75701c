import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: long CPU test")


@pytest.fixture(scope="session")
def O():
    from oracle import oracle
    oracle.lib()
    return oracle


@pytest.fixture(scope="session")
def ctx():
    """One device context for the GPU tests: a 64 GiB torch arena on cuda:0."""
    import torch

    import paper_2512_04216_amd as S

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    c = S.Context(arena_bytes=64 << 30, device=0, renorm_period=64)
    yield c
    c.close()


@pytest.fixture(scope="session")
def S():
    import paper_2512_04216_amd as S

    S.load()
    return S


def infidelity(a, b):
    import numpy as np

    a = np.asarray(a, dtype=np.complex128)
    b = np.asarray(b, dtype=np.complex128)
    ov = np.vdot(a, b)
    return float(1.0 - abs(ov) ** 2 / (np.vdot(a, a).real * np.vdot(b, b).real))
