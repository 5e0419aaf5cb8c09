import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line('markers', 'gpu: needs an MI355X (runs the HIP library through the C ABI)')


@pytest.fixture(scope='session')
def orc():
    from oracle import native
    native.lib()
    return native


TESTS = os.path.dirname(os.path.abspath(__file__))
if TESTS not in sys.path:
    sys.path.insert(0, TESTS)


@pytest.fixture(scope='session')
def gpu():
    """The HIP library on cuda:0 (the test is marked gpu; no CPU fallback exists)."""
    import torch
    import paper_2509_05464_amd as fq
    assert torch.cuda.is_available(), 'GPU tests need an MI355X'
    fq.lib()
    return fq
